"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/escg.h, and its host-side parameter preparation (dominance
bitmasks, action thresholds, validation) agrees with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd import escg, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "escg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(escg_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("escg_init", "escg_step_mcs", "escg_densities",
              "escg_run_until_extinction", "escg_batch_run"):
        assert n in names
    assert set(names) == set(escg.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = escg.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_status_strings():
    assert escg.status_str(0) == "ok"
    assert escg.status_str(-1) == "invalid argument"


@pytest.mark.parametrize("S,K", [(3, [1]), (5, [1, 3]), (5, [1, 2]),
                                 (8, [1, 2, 5]), (31, [1, 7, 30]), (1, [])])
def test_dominance_bitmasks_match_oracle_matrix(S, K):
    D = O.circulant_matrix(S, K) if K else np.zeros((S, S), np.uint8)
    dom = escg.circulant_dom(S, K)
    assert dom == escg.dom_from_matrix(D)
    for a in range(1, S + 1):
        for b in range(1, S + 1):
            assert ((dom[a] >> b) & 1) == D[a - 1, b - 1]
    assert dom[0] == 0 and all((d & 1) == 0 for d in dom)


@pytest.mark.parametrize("rates", [(0.5, 1, 1), (13.1072, 1, 1), (51.2, 1, 1),
                                   (0, 1, 1), (1, 0, 1), (1, 1, 0), (3, 2, 5),
                                   (1e-9, 1, 1), (1280.0, 1, 1)])
def test_thresholds_match_oracle(rates):
    p = escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=rates[0],
                    sel=rates[1], rep=rates[2])
    assert escg.thresholds(p) == O.thresholds(*rates)


@pytest.mark.parametrize("M,L,eps", [(1e-5, 3200, 51.2), (1e-4, 512, 13.1072),
                                     (1e-3, 64, 2.048), (0.0, 100, 0.0)])
def test_eps_from_mobility_is_the_workload_convention(M, L, eps):
    # M = 2 eps / N with N = L^2 sites; the workload tables quote these eps
    assert escg.eps_from_mobility(M, L) == pytest.approx(eps, rel=1e-12)
    assert escg.eps_from_mobility(M, L) == workloads.eps_from_mobility(M, L)


@pytest.mark.parametrize("M,L", [(-1e-5, 64), (float("nan"), 64),
                                 (float("inf"), 64), (1e-5, 0)])
def test_eps_from_mobility_rejects_bad_input(M, L):
    with pytest.raises(escg.EscgError):
        escg.eps_from_mobility(M, L)


def _bad_params():
    good = dict(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1.0)
    yield dict(good, L=7)
    yield dict(good, L=0)
    yield dict(good, L=46342)
    yield dict(good, S=0)
    yield dict(good, S=32)
    yield dict(good, ex=-1.0)
    yield dict(good, ex=float("nan"))
    yield dict(good, ex=float("inf"))
    yield dict(good, ex=0.0, sel=0.0, rep=0.0)
    yield dict(good, dom=[1] + [0] * 31)            # dom[0] set
    yield dict(good, dom=[0, 1 << 5] + [0] * 30)    # bit above S
    yield dict(good, dom=[0, 1] + [0] * 30)         # bit 0 set
    yield dict(good, dom=[0, 2, 4, 8, 2] + [0] * 27)  # species 4 > S


@pytest.mark.parametrize("kw", list(_bad_params()))
def test_invalid_params_rejected_before_any_device_work(kw):
    p = escg.Params(**kw).c()
    lib = escg.lib()
    dummy = C.c_void_p(4096)  # never dereferenced: validation fails first
    res = C.c_void_p(8192)
    assert lib.escg_init(C.byref(p), dummy, None) == escg.EINVAL
    assert lib.escg_step_mcs(C.byref(p), dummy, 0, 1, None, None) == escg.EINVAL
    assert lib.escg_densities(C.byref(p), dummy, res, None) == escg.EINVAL
    assert lib.escg_run_until_extinction(C.byref(p), dummy, 0, 1, 0, res,
                                         None) == escg.EINVAL


def test_null_and_misaligned_pointers_rejected():
    p = escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1.0).c()
    lib = escg.lib()
    assert lib.escg_init(C.byref(p), None, None) == escg.EINVAL
    assert lib.escg_init(C.byref(p), C.c_void_p(4097), None) == escg.EINVAL
    assert lib.escg_densities(C.byref(p), C.c_void_p(4096), None,
                              None) == escg.EINVAL
    assert lib.escg_run_until_extinction(C.byref(p), C.c_void_p(4096), 0, 1,
                                         7, C.c_void_p(64), None) == escg.EINVAL
    assert lib.escg_init(None, C.c_void_p(4096), None) == escg.EINVAL


def test_batch_rejects_overlap_and_bad_jobs():
    lib = escg.lib()
    P = escg.CParams * 2
    ps = P(escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1).c(),
           escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1).c())
    mx = (C.c_uint32 * 2)(5, 5)
    overl = (C.c_uint64 * 2)(0, 32)   # second lattice starts inside the first
    assert lib.escg_batch_run(2, ps, overl, C.c_void_p(4096), None, mx, 0, 1,
                              C.c_void_p(8192), None) == escg.EINVAL
    mis = (C.c_uint64 * 2)(0, 66)     # not 4-byte aligned
    assert lib.escg_batch_run(2, ps, mis, C.c_void_p(4096), None, mx, 0, 1,
                              C.c_void_p(8192), None) == escg.EINVAL
    ok = (C.c_uint64 * 2)(0, 64)
    assert lib.escg_batch_run(2, ps, ok, C.c_void_p(4096), None, mx, 9, 1,
                              C.c_void_p(8192), None) == escg.EINVAL
    assert lib.escg_batch_run(0, None, None, None, None, None, 0, 1, None,
                              None) == escg.OK
    # an empty step batch is a no-op too (nothing touches the device)
    assert lib.escg_step_batch(0, None, None, None, None, None) == escg.OK
    assert lib.escg_step_batch(1, None, None, None, None, None) == escg.EINVAL


@pytest.mark.parametrize("flags", [2, 4, 0x80000000, 3])
def test_unknown_flag_bits_rejected(flags):
    cp = escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1.0).c()
    cp.flags = flags
    # validation precedes any device work: a fake (aligned) pointer is safe
    assert escg.lib().escg_step_mcs(C.byref(cp), C.c_void_p(4096), 0, 1,
                                    None, None) == escg.EINVAL


@pytest.mark.parametrize("bad", [-0.1, 1.5, float("nan"), float("inf")])
def test_dominance_probabilities_outside_unit_interval_rejected(bad):
    D = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], np.uint8)
    P = D * 0.5
    P[1, 0] = bad   # even where D has no edge: every entry must be in [0, 1]
    cp = escg.Params(L=8, S=3, dom=escg.dom_from_matrix(D), ex=1.0,
                     prob=P).c()
    assert escg.lib().escg_step_mcs(C.byref(cp), C.c_void_p(4096), 0, 1,
                                    None, None) == escg.EINVAL


def test_moore_flag_is_bit_zero():
    assert escg.FLAG_MOORE == 1
    cp = escg.Params(L=8, S=3, dom=escg.circulant_dom(3, [1]), ex=1.0,
                     moore=True).c()
    assert cp.flags == 1
    src = open(os.path.join(ROOT, "include", "escg.h")).read()
    assert re.search(r"#define ESCG_FLAG_MOORE 1u", src)


def test_launch_choices_travel_in_params():
    # per-call launch choices: route, tile shape, thread cap, workgroups per
    # CU; the library exports no process-wide routing setters
    p = escg.Params(L=3200, S=5, dom=escg.circulant_dom(5, [1, 3]), ex=51.2)
    c = p.c()
    assert (c.launch.route, c.launch.tile_h, c.launch.tile_w,
            c.launch.threads, c.launch.wg_per_cu) == (0, 0, 0, 0, 0)
    q = p.with_launch(route="persistent", tile=(100, 400), threads=768,
                      wg_per_cu=2, max_wgs=192).c()
    assert (q.launch.route, q.launch.tile_h, q.launch.tile_w,
            q.launch.threads, q.launch.wg_per_cu,
            q.launch.max_wgs) == (3, 100, 400, 768, 2, 192)
    # the binding's struct has the header's six launch fields, in order
    src = open(os.path.join(ROOT, "include", "escg.h")).read()
    body = src[src.index("typedef struct escg_launch {"):
               src.index("} escg_launch;")]
    fields = re.findall(r"uint32_t ([a-z_, ]+);", body)
    names = [n.strip() for f in fields for n in f.split(",")]
    assert names == [f for f, _ in escg.CLaunch._fields_]
    assert p.route == "auto"                      # p itself is unchanged
    L = escg.lib()
    for name in ("escg_set_single_lds_max_L", "escg_set_persistent_min_L",
                 "escg_set_tile_shape"):
        assert not hasattr(L, name), name
    src = open(os.path.join(ROOT, "include", "escg.h")).read()
    assert "escg_launch launch;" in src


@pytest.mark.parametrize("field,value", [("route", 4), ("threads", 96),
                                         ("threads", 2048), ("wg_per_cu", 9),
                                         ("tile_h", 3)])
def test_invalid_launch_choices_rejected_before_device_work(field, value):
    p = escg.Params(L=3200, S=5, dom=escg.circulant_dom(5, [1, 3]), ex=51.2)
    c = p.c()
    if field == "tile_h":
        c.launch.tile_h, c.launch.tile_w = value, 400
    else:
        setattr(c.launch, field, value)
    # a bogus device pointer: validation must fail before any use of it
    s = escg.lib().escg_step_mcs(C.byref(c), C.c_void_p(0x1000), 0, 1, None,
                                 None)
    assert s == escg.EINVAL


def test_batch_limits_callable_without_gpu():
    assert escg.batch_max_L(0) == 0 and escg.batch_max_L(32) == 0
    assert escg.batch_max_L(3) >= escg.batch_max_L(31) > 0


def test_tile_plan_kind_checked_before_device_work():
    p = escg.Params(L=1600, S=3, dom=escg.circulant_dom(3, [1]), ex=1.0).c()
    a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
    assert escg.lib().escg_tile_plan(C.byref(p), 3, C.byref(a), C.byref(b),
                                     C.byref(c)) == escg.EINVAL
