"""The job server on the GPU: every job's final lattice and counts are
byte-identical to the same job run alone (and to the oracle for the cheap
ones), with small jobs batched in one launch and large jobs overlapping on
their own streams."""
import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd import escg
from paper_2508_16639_amd.serve import DeviceExecutor, Scheduler, ServerConfig
from paper_2508_16639_amd.workloads import Request

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def requests(n=30, seed=7):
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(n):
        t += rng.exponential(0.004)
        S, K = ((3, (1,)) if rng.random() < 0.5 else (5, (1, 3)))
        L = int(rng.choice([32, 64, 100, 200, 400, 800]))
        M = float(10 ** rng.uniform(-6, -3))
        out.append(Request(job_id=i, arrival_s=t, L=L, S=S, K=K, M=M,
                           ex=M * L * L / 2, mcs=int(rng.integers(5, 60)),
                           seed=1000 + i))
    return out


def alone_gpu(r):
    p = escg.Params(L=r.L, S=r.S, dom=escg.circulant_dom(r.S, r.K), ex=r.ex,
                    seed=r.seed)
    lat = torch.empty(r.L * r.L, dtype=torch.uint8, device="cuda")
    escg.init(p, lat)
    escg.step_mcs(p, lat, 0, r.mcs, None)
    torch.cuda.synchronize()
    return lat.cpu().numpy()


@pytest.mark.parametrize("large_route", ["persistent", "tiled"])
def test_server_results_equal_alone_runs(large_route):
    reqs = requests()
    ex = DeviceExecutor(torch, escg, keep_lattices=True,
                        large_route=large_route)
    st, jobs = Scheduler(ex, ServerConfig(work_per_iter=2e6,
                                          min_chunk=3)).run(reqs)
    escg.async_status()
    assert st.completed == len(reqs) and st.failed == 0
    assert st.iterations > 1 and st.peak_active > 1
    for r in reqs:
        got = ex.final_lattices[r.job_id]
        assert np.array_equal(got, alone_gpu(r)), r.job_id
        assert np.array_equal(jobs[r.job_id].result,
                              np.bincount(got, minlength=r.S + 1))
    for r in [r for r in reqs if r.L * r.L * r.mcs < 3e6][:5]:
        j = O.Job(r.L, r.S, O.circulant_matrix(r.S, r.K), r.ex, seed=r.seed)
        g = j.init()
        O.o2_run(j, g, 0, r.mcs, want_counts=False)
        assert np.array_equal(ex.final_lattices[r.job_id], g)


def test_server_under_small_hbm_budget_queues_instead_of_dropping():
    reqs = requests(16, seed=9)
    ex = DeviceExecutor(torch, escg)
    cfg = ServerConfig(hbm_budget=2 * 2 * 800 * 800 + 3 * 4096,
                       work_per_iter=2e6, min_chunk=3)
    st, jobs = Scheduler(ex, cfg).run(reqs)
    assert st.completed == len(reqs) and st.failed == 0
    assert st.peak_footprint <= cfg.hbm_budget


def test_server_mixes_wide_and_narrow_species_tables():
    """Small jobs with S > 7 (wide rule tables, a smaller LDS limit) and
    S <= 7 at L = 400 in the same iterations, beside large jobs (L = 800,
    1600) in persistent launches: each result equals the job alone."""
    reqs = []
    for i, (L, S, K) in enumerate([(400, 3, (1,)), (256, 13, (1, 2, 5)),
                                   (400, 5, (1, 3)), (1600, 5, (1, 3)),
                                   (200, 13, (1, 2, 5)), (800, 3, (1,)),
                                   (400, 3, (1,)), (1600, 3, (1,))]):
        M = 10.0 ** (-3 - i % 3)
        reqs.append(Request(job_id=i, arrival_s=0.002 * i, L=L, S=S, K=K,
                            M=M, ex=M * L * L / 2, mcs=9 + 5 * i,
                            seed=300 + i))
    ex = DeviceExecutor(torch, escg, keep_lattices=True)
    st, jobs = Scheduler(ex, ServerConfig(work_per_iter=4e7,
                                          min_chunk=4)).run(reqs)
    escg.async_status()
    assert st.completed == len(reqs) and st.failed == 0
    for r in reqs:
        assert np.array_equal(ex.final_lattices[r.job_id], alone_gpu(r)), \
            r.job_id
