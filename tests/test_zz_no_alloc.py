"""The entry point that allocates nothing (escg_step_mcs_static), called
through the C ABI: on every route it gives the bytes and counts of
escg_step_mcs, on two calls in a row (the second on a smaller job, so the
shared static array keeps the first call's contents), and it rejects a job
whose scratch would exceed the array with nothing enqueued."""
import ctypes as C

import numpy as np
import pytest

from paper_2508_16639_amd import escg
from paper_2508_16639_amd.workloads import random_lattice
from tests.gpu_util import dev, host, pair, probabilities

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(fn_name, p, g0, mcs0, n):
    lat = dev(g0)
    cnt = torch.full(((n + 1) * (p.S + 1),), -1, dtype=torch.int32,
                     device="cuda:0")
    cp = p.c()
    s = getattr(escg.lib(), fn_name)(
        C.byref(cp), C.c_void_p(lat.data_ptr()), mcs0, n,
        C.c_void_p(cnt.data_ptr()),
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert s == escg.OK, (fn_name, s, escg.last_error())
    route = escg.last_route()
    return host(lat), host(cnt), route


# (first job, second smaller job) per route: L, S, K, ex, n_mcs, probabilities
CASES = {
    "persistent": [(512, 5, [1, 3], 13.1, 6, False),
                   (136, 3, [1], 2.0, 4, True)],
    "tiled": [(520, 8, [1, 3], 5.0, 3, False), (200, 5, [1, 3], 1.0, 2, True)],
    "lds": [(256, 5, [1, 3], 3.0, 5, True), (64, 3, [1], 0.5, 7, False)],
}


@pytest.mark.parametrize("route", list(CASES))
def test_static_scratch_equals_step_mcs_twice(route):
    for i, (L, S, K, ex, n, prob) in enumerate(CASES[route]):
        D = None
        P = None
        if prob:
            from oracle import circulant_matrix
            D = circulant_matrix(S, K)
            P = probabilities(D, seed=L)
        p, _ = pair(L, S, K if D is None else None, ex, seed=40 + i,
                    replica=i, D=D, P=P, route=route)
        g0 = random_lattice(L, S, seed=L + i, domain=3)
        a, ca, ra = _run("escg_step_mcs", p, g0, 11, n)
        b, cb, rb = _run("escg_step_mcs_static", p, g0, 11, n)
        assert ra == rb == route, (ra, rb)
        assert np.array_equal(a, b), (route, L)
        assert np.array_equal(ca, cb), (route, L)


def test_static_scratch_rejects_oversize_job_with_nothing_enqueued():
    L = 8200                              # per-MCS path: L*L > 64 MiB
    p, _ = pair(L, 3, [1], 1.0, route="tiled")
    lat = torch.zeros(L * L, dtype=torch.uint8, device="cuda:0")
    cnt = torch.full((2 * 4,), -1, dtype=torch.int32, device="cuda:0")
    cp = p.c()
    s = escg.lib().escg_step_mcs_static(
        C.byref(cp), C.c_void_p(lat.data_ptr()), 0, 1,
        C.c_void_p(cnt.data_ptr()),
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert s == escg.ENOMEM
    assert "static scratch" in escg.last_error()
    torch.cuda.synchronize()
    assert int(lat.sum()) == 0
    assert (host(cnt) == 0xFFFFFFFF).all()
