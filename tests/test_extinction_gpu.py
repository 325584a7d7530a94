"""Parity of the stop-condition runner and of the batched persistent kernel
with the oracle: flag, stop time, final counts and final lattice."""
import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd import escg
from paper_2508_16639_amd.workloads import batch_replicas, random_lattice
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MODES = [escg.STOP_FIRST_EXTINCTION, escg.STOP_MONOCULTURE, escg.STOP_NONE]


def oracle_until(j, g, mcs0, cap, mode):
    if mode == escg.STOP_NONE:
        c = O.o2_run(j, g, mcs0, cap)
        return np.concatenate([[0, cap], c[-1]]).astype(np.uint32)
    return O.o2_run_until(j, g, mcs0, cap, mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,S,K,ex,cap", [
    (8, 3, [1], 2.0, 300), (16, 3, [1], 4.0, 400), (32, 5, [1, 3], 3.0, 150),
    (64, 3, [1], 1.0, 60), (100, 3, [1], 20.0, 40), (404, 3, [1], 50.0, 3),
    (416, 3, [1], 50.0, 3), (24, 2, [1], 1.0, 200)])
def test_run_until_bit_exact(mode, L, S, K, ex, cap):
    hits = 0
    for rep in range(3):
        p, j = pair(L, S, K, ex, seed=77, replica=rep)
        g0 = j.init()
        lat = dev(g0)
        res = torch.full((S + 3,), -1, dtype=torch.int32, device="cuda:0")
        escg.run_until_extinction(p, lat, 5, cap, mode, res)
        ref = g0.copy()
        r = oracle_until(j, ref, 5, cap, mode)
        got = host(res)
        assert np.array_equal(got, r), (rep, got, r)
        assert np.array_equal(host(lat), ref)
        hits += int(r[0])
    if mode == escg.STOP_NONE:
        assert hits == 0


def test_run_until_input_already_met():
    p, j = pair(64, 3, [1], 1.0)
    g = np.zeros(64 * 64, np.uint8)
    g[:10] = 2
    res = torch.full((6,), -1, dtype=torch.int32, device="cuda:0")
    lat = dev(g)
    escg.run_until_extinction(p, lat, 0, 100, escg.STOP_FIRST_EXTINCTION, res)
    assert host(res).tolist() == [1, 0, 64 * 64 - 10, 0, 10, 0]
    assert np.array_equal(host(lat), g)


# species 1 beats 2 and 3, which do not interact: 1 takes over, at times
# (weak selection) that fall in the second to fifth chunk of the persistent
# runner (chunks of 64, 128, 256, 512, 1024 MCS)
D_TAKEOVER = np.array([[0, 1, 1], [0, 0, 0], [0, 0, 0]], np.uint8)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("L,ex,sel,cap", [(80, 0.5, 1.0, 200),
                                          (80, 0.5, 0.03, 3000),
                                          (96, 1.0, 0.01, 3000)])
def test_run_until_persistent_chunks_stop_exactly(mode, L, ex, sel, cap):
    cap = cap if mode != escg.STOP_NONE else 150
    for rep in range(2):
        p, j = pair(L, 3, None, ex, sel, 1.0, seed=77, replica=rep,
                    D=D_TAKEOVER)
        g0 = j.init()
        lat = dev(g0)
        res = torch.full((6,), -1, dtype=torch.int32, device="cuda:0")
        escg.run_until_extinction(p, lat, 5, cap, mode, res)
        assert escg.last_route() == "persistent", escg.last_error()
        ref = g0.copy()
        r = oracle_until(j, ref, 5, cap, mode)
        assert np.array_equal(host(res), r), (rep, host(res), r)
        assert np.array_equal(host(lat), ref)
        if mode != escg.STOP_NONE:
            assert r[0] == 1


def test_run_until_persistent_input_already_met():
    p, j = pair(96, 3, [1], 1.0)
    g = np.zeros(96 * 96, np.uint8)
    g[:10] = 2
    res = torch.full((6,), -1, dtype=torch.int32, device="cuda:0")
    lat = dev(g)
    escg.run_until_extinction(p, lat, 0, 100, escg.STOP_FIRST_EXTINCTION, res)
    assert escg.last_route() == "persistent"
    assert host(res).tolist() == [1, 0, 96 * 96 - 10, 0, 10, 0]
    assert np.array_equal(host(lat), g)


def _batch(jobs, mode, init, mcs0=None):
    """jobs: list of (Params, oracle Job, cap, g0 or None)."""
    offs, off = [], 0
    for p, _, _, _ in jobs:
        offs.append(off)
        off += (p.L * p.L + 255) // 256 * 256
    buf = torch.zeros(off, dtype=torch.uint8, device="cuda:0")
    for (p, _, _, g0), o in zip(jobs, offs):
        if g0 is not None:
            buf[o:o + p.L * p.L] = dev(g0)
    res = torch.full((len(jobs) * escg.BATCH_RESULT_WORDS,), -1,
                     dtype=torch.int32, device="cuda:0")
    escg.batch_run([x[0] for x in jobs], offs, buf, [x[2] for x in jobs],
                   mode, init, res, mcs0=mcs0)
    out = host(buf)
    r = host(res).reshape(len(jobs), escg.BATCH_RESULT_WORDS)
    lats = [out[o:o + p.L * p.L] for (p, _, _, _), o in zip(jobs, offs)]
    return lats, r


@pytest.mark.parametrize("mode", MODES)
def test_batch_equals_oracle_mixed_sizes(mode):
    rng = np.random.default_rng(4)
    jobs = []
    for i in range(40):
        L = int(rng.choice([4, 8, 16, 30, 64, 96, 130]))
        S, K = ((3, [1]) if i % 3 else (5, [1, 3]))
        ex = float(10 ** rng.uniform(-1, 1.5))
        cap = int(rng.integers(0, 60))
        p, j = pair(L, S, K, ex, seed=1000 + i, replica=i)
        jobs.append((p, j, cap, None))
    mcs0 = [int(x) for x in rng.integers(0, 1000, size=len(jobs))]
    lats, r = _batch(jobs, mode, True, mcs0)
    for (p, j, cap, _), lat, rr, m0 in zip(jobs, lats, r, mcs0):
        g = j.init()
        ref = oracle_until(j, g, m0, cap, mode)
        assert np.array_equal(rr[:p.S + 3], ref), (p.L, cap)
        assert (rr[p.S + 3:] == 0).all()
        assert np.array_equal(lat, g)


def test_batch_given_lattices_and_dominance_table_path():
    # S = 9 > 7 uses the LDS dominance-table instantiation
    jobs = []
    for i in range(6):
        L = 32 + 16 * i
        p, j = pair(L, 9, [1, 2, 4], 1.5, seed=3, replica=i)
        jobs.append((p, j, 25, random_lattice(L, 9, seed=i, domain=2)))
    lats, r = _batch(jobs, escg.STOP_MONOCULTURE, False)
    for (p, j, cap, g0), lat, rr in zip(jobs, lats, r):
        g = g0.copy()
        ref = O.o2_run_until(j, g, 0, cap, O.MONOCULTURE)
        assert np.array_equal(rr[:p.S + 3], ref)
        assert np.array_equal(lat, g)


def test_batch_equals_single_calls_on_gpu():
    jobs = []
    for i in range(12):
        L = [64, 128, 192, 256][i % 4]
        p, j = pair(L, 3, [1], float(10 ** (-1 + i / 4)), seed=1, replica=i)
        jobs.append((p, j, 30, None))
    lats, r = _batch(jobs, escg.STOP_FIRST_EXTINCTION, True)
    for (p, j, cap, _), lat, rr in zip(jobs, lats, r):
        one = torch.empty(p.L * p.L, dtype=torch.uint8, device="cuda:0")
        escg.init(p, one)
        res = torch.empty(p.S + 3, dtype=torch.int32, device="cuda:0")
        escg.run_until_extinction(p, one, 0, cap, escg.STOP_FIRST_EXTINCTION,
                                  res)
        assert np.array_equal(host(one), lat)
        assert np.array_equal(host(res), rr[:p.S + 3])


def test_batch_workload_full_size_sampled():
    """The 4,096-replica extinction workload in the benchmark's launch
    configuration; replicas the oracle can redo quickly are checked one by
    one, the rest by invariants."""
    tab = batch_replicas()
    n = len(tab)
    params, offs, off = [], [], 0
    for r in range(n):
        L = int(tab.L[r])
        params.append(escg.Params(L=L, S=3, dom=escg.circulant_dom(3, [1]),
                                  ex=float(tab.ex[r]), seed=tab.seed,
                                  replica=r))
        offs.append(off)
        off += L * L
    buf = torch.empty(off, dtype=torch.uint8, device="cuda:0")
    res = torch.empty(n * escg.BATCH_RESULT_WORDS, dtype=torch.int32,
                      device="cuda:0")
    escg.batch_run(params, offs, buf, tab.max_mcs, escg.STOP_FIRST_EXTINCTION,
                   True, res)
    r = host(res).reshape(n, escg.BATCH_RESULT_WORDS)
    out = host(buf)
    L2 = tab.L.astype(np.int64) ** 2
    assert (r[:, 1] <= tab.max_mcs).all()
    assert (r[:, 2:6].sum(1) == L2).all()
    ext = r[:, 0] == 1
    assert ((r[ext, 3:6] == 0).any(1)).all()
    assert ((r[~ext, 1] == tab.max_mcs[~ext])).all()
    cost = L2 * np.maximum(r[:, 1], 1)
    sample = list(np.argsort(cost)[:6]) + [int(np.argmax(tab.L == 256))]
    for i in sample:
        L = int(tab.L[i])
        j = O.Job(L, 3, O.circulant_matrix(3, [1]), float(tab.ex[i]),
                  seed=tab.seed, replica=int(i))
        g = j.init()
        cap = int(min(tab.max_mcs[i], r[i, 1] if r[i, 0] else 30))
        if cap < tab.max_mcs[i] and not r[i, 0]:
            continue
        ref = O.o2_run_until(j, g, 0, int(tab.max_mcs[i]) if r[i, 0] else cap,
                             O.FIRST_EXTINCTION)
        if r[i, 0]:
            assert np.array_equal(r[i, :6], ref)
            assert np.array_equal(out[offs[i]:offs[i] + L * L], g)
