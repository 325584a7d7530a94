"""Scheduler logic of the job server on the CPU: admission under an HBM
budget and slot limit, no dropped jobs, latency accounting, failure
isolation, and results independent of co-runners and chunking."""
import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd.serve import (Scheduler, ServerConfig,
                                        footprint_bytes)
from paper_2508_16639_amd.workloads import Request, serving_requests
from tests.serve_fakes import FakeClock, OracleExecutor


def small_requests(n=24, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(0.01)
        S, K = ((3, (1,)) if i % 2 else (5, (1, 3)))
        L = int(rng.choice([8, 12, 16, 24]))
        out.append(Request(job_id=i, arrival_s=t, L=L, S=S, K=K, M=1e-3,
                           ex=float(rng.uniform(0.1, 3.0)),
                           mcs=int(rng.integers(5, 40)), seed=100 + i))
    return out


def alone(req):
    j = O.Job(req.L, req.S, O.circulant_matrix(req.S, req.K), req.ex, 1.0,
              1.0, seed=req.seed)
    g = j.init()
    O.o2_run(j, g, 0, req.mcs, want_counts=False)
    return g


def run(reqs, cfg, **kw):
    clock = FakeClock()
    ex = OracleExecutor(clock, **kw)
    st, jobs = Scheduler(ex, cfg, clock=clock, sleep=clock.sleep).run(reqs)
    return st, jobs, ex


def test_every_job_completes_and_matches_alone_run():
    reqs = small_requests()
    cfg = ServerConfig(hbm_budget=10**9, max_active=6, work_per_iter=3000,
                       min_chunk=1, max_chunk=7)
    st, jobs, ex = run(reqs, cfg)
    assert st.completed == len(reqs) and st.failed == 0
    assert st.iterations > len(reqs) // 6
    for r in reqs:
        assert np.array_equal(ex.final[r.job_id], alone(r)), r.job_id
        assert np.array_equal(jobs[r.job_id].result,
                              O.counts(alone(r), r.L, r.S))


def test_admission_respects_budget_and_slots_and_never_drops():
    reqs = small_requests(30)
    budget = 3 * footprint_bytes(24)
    cfg = ServerConfig(hbm_budget=budget, max_active=2, work_per_iter=2000,
                       min_chunk=1)
    st, jobs, ex = run(reqs, cfg)
    assert st.completed == len(reqs)
    assert st.peak_footprint <= budget
    assert st.peak_active <= 2 and ex.max_live <= 2
    # FIFO admission: admission times follow arrival order
    adm = [jobs[r.job_id].t_admit for r in sorted(reqs,
                                                  key=lambda r: r.arrival_s)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_latency_is_completion_minus_arrival():
    reqs = small_requests(10)
    cfg = ServerConfig(hbm_budget=10**9, work_per_iter=1e6)
    st, jobs, _ = run(reqs, cfg, su_per_s=1e6)
    for r in reqs:
        js = jobs[r.job_id]
        assert js.t_done >= r.arrival_s
        assert js.t_admit >= r.arrival_s
    lat = sorted(jobs[r.job_id].t_done - r.arrival_s for r in reqs)
    assert sorted(st.latencies) == pytest.approx(lat)
    s = st.summary()
    assert s["p50_latency_s"] <= s["p99_latency_s"]
    assert s["jobs_per_s"] == pytest.approx(len(reqs) / st.wall)


def test_invalid_and_oversized_jobs_are_isolated():
    reqs = small_requests(12)
    bad = reqs[3]
    reqs[3] = Request(job_id=bad.job_id, arrival_s=bad.arrival_s, L=7,
                      S=3, K=(1,), M=1e-3, ex=1.0, mcs=10, seed=1)
    big = reqs[5]
    reqs[5] = Request(job_id=big.job_id, arrival_s=big.arrival_s, L=64,
                      S=3, K=(1,), M=1e-3, ex=1.0, mcs=10, seed=1)
    cfg = ServerConfig(hbm_budget=footprint_bytes(32), work_per_iter=2000)
    st, jobs, ex = run(reqs, cfg, fail_on={7})
    assert st.failed == 3
    assert "rejected" in jobs[3].failed and "rejected" in jobs[7].failed
    assert "budget" in jobs[5].failed
    for r in reqs:
        if r.job_id in (3, 5, 7):
            continue
        assert np.array_equal(ex.final[r.job_id], alone(r))


def test_executor_failure_fails_that_iteration_and_continues():
    reqs = small_requests(16)
    cfg = ServerConfig(hbm_budget=10**9, max_active=4, work_per_iter=1500,
                       min_chunk=1)
    st, jobs, ex = run(reqs, cfg, fail_iter=3)
    assert st.failed >= 1 and st.completed + st.failed == len(reqs)
    for r in reqs:
        if not jobs[r.job_id].failed:
            assert np.array_equal(ex.final[r.job_id], alone(r))


def test_serving_workload_recipe():
    reqs = serving_requests(n=500)
    gaps = np.diff([r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 1 / 200) < 0.0015
    assert {r.L for r in reqs} == {100, 200, 400, 800, 1600}
    assert {r.S for r in reqs} == {3, 5}
    assert min(r.mcs for r in reqs) >= 500 and max(r.mcs for r in reqs) <= 5000
    for r in reqs:
        assert r.ex == pytest.approx(r.M * r.L * r.L / 2)
