"""Python binding of the ESCG C ABI (``include/escg.h``).

Argument marshalling only: every step of the path runs in the HIP library.
Device buffers are torch tensors on the current device; work is enqueued on
torch's current stream (or an explicit ``stream``) and is asynchronous.
There is no CPU fallback: if ``libescg.so`` is missing or fails to load,
``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
import dataclasses
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                         "libescg.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ETIMEOUT = 0, -1, -2, -3, -4, -5
ROUTE_LDS, ROUTE_TILED, ROUTE_PERSISTENT = 1, 2, 3
ROUTE_NAMES = {0: "none", 1: "lds", 2: "tiled", 3: "persistent"}
ROUTE_CODES = {"auto": 0, "lds": 1, "tiled": 2, "persistent": 3}
STOP_FIRST_EXTINCTION, STOP_MONOCULTURE, STOP_NONE = 0, 1, 2
BATCH_RESULT_WORDS = 34
FLAG_MOORE = 1           # ESCG_FLAG_MOORE: 8-way neighbourhood
MAX_SPECIES = 31


class EscgError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = f"{what}: {status_str(status)} ({status})"
        if status == EDEVICE:
            msg += f" [{lib().escg_last_error().decode()}]"
        super().__init__(msg)
        self.status = status


class CLaunch(C.Structure):
    _fields_ = [("route", C.c_uint32), ("tile_h", C.c_uint32),
                ("tile_w", C.c_uint32), ("threads", C.c_uint32),
                ("wg_per_cu", C.c_uint32), ("max_wgs", C.c_uint32)]


class CParams(C.Structure):
    _fields_ = [("L", C.c_uint32), ("S", C.c_uint32),
                ("dom", C.c_uint32 * 32),
                ("rate_ex", C.c_double), ("rate_sel", C.c_double),
                ("rate_rep", C.c_double), ("seed", C.c_uint64),
                ("replica", C.c_uint32), ("flags", C.c_uint32),
                ("dom_prob", C.c_void_p), ("launch", CLaunch)]


STATIC_SCRATCH_BYTES = 64 << 20   # ESCG_STATIC_SCRATCH_BYTES
EXPORTS = ("escg_status_str", "escg_last_error", "escg_circulant_dom", "escg_dom_from_matrix",
           "escg_thresholds", "escg_eps_from_mobility", "escg_init", "escg_densities", "escg_step_mcs",
           "escg_run_until_extinction", "escg_batch_max_L", "escg_batch_run",
           "escg_step_batch", "escg_async_status", "escg_last_route",
           "escg_tile_plan", "escg_step_mcs_static")

_lib = None


def lib():
    """Loads libescg.so (built by ``__graft_entry__.build()``); raises if it
    is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is not built; run __graft_entry__.build() first")
    # torch ships its own HIP runtime (same soname as /opt/rocm's); loading it
    # first makes the library bind to that one, so device pointers and
    # streams are shared with torch instead of living in a second runtime.
    import torch  # noqa: F401
    L = C.CDLL(_LIB_PATH)
    P = C.POINTER(CParams)
    u32p = C.POINTER(C.c_uint32)
    vp = C.c_void_p
    u32 = C.c_uint32
    L.escg_status_str.argtypes = [C.c_int32]
    L.escg_status_str.restype = C.c_char_p
    L.escg_last_error.argtypes = []
    L.escg_last_error.restype = C.c_char_p
    L.escg_circulant_dom.argtypes = [u32, u32, u32p]
    L.escg_dom_from_matrix.argtypes = [u32, C.POINTER(C.c_uint8), u32p]
    L.escg_thresholds.argtypes = [P, u32p, u32p]
    L.escg_eps_from_mobility.argtypes = [C.c_double, u32,
                                         C.POINTER(C.c_double)]
    L.escg_init.argtypes = [P, vp, vp]
    L.escg_densities.argtypes = [P, vp, vp, vp]
    L.escg_step_mcs.argtypes = [P, vp, u32, u32, vp, vp]
    L.escg_step_mcs_static.argtypes = [P, vp, u32, u32, vp, vp]
    L.escg_run_until_extinction.argtypes = [P, vp, u32, u32, u32, vp, vp]
    L.escg_batch_max_L.argtypes = [u32]
    L.escg_batch_max_L.restype = u32
    L.escg_batch_run.argtypes = [u32, P, C.POINTER(C.c_uint64), vp,
                                 u32p, u32p, u32, u32, vp, vp]
    L.escg_step_batch.argtypes = [u32, P, C.POINTER(C.c_void_p), u32p,
                                  u32p, vp]
    L.escg_async_status.argtypes = [C.c_int]
    L.escg_tile_plan.argtypes = [P, u32, u32p, u32p, u32p]
    L.escg_last_route.argtypes = []
    L.escg_last_route.restype = u32
    for name in EXPORTS:
        if name not in ("escg_status_str", "escg_batch_max_L",
                        "escg_last_error", "escg_last_route"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def status_str(s: int) -> str:
    return lib().escg_status_str(int(s)).decode()


def _check(status: int, what: str):
    if status != OK:
        raise EscgError(status, what)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

@dataclass
class Params:
    """Job parameters.  ``dom`` is 32 uint32 bitmasks (see escg.h); build it
    with :func:`circulant_dom` or :func:`dom_from_matrix`."""
    L: int
    S: int
    dom: Sequence[int]
    ex: float
    sel: float = 1.0
    rep: float = 1.0
    seed: int = 1
    replica: int = 0
    moore: bool = False      # 8-way (Moore) instead of 4-way neighbourhood
    prob: Optional[object] = None  # S x S dominance probabilities or None
    # launch choices (escg_launch; all default: the library decides)
    route: str = "auto"      # "auto", "lds", "tiled" or "persistent"
    tile: Optional[Tuple[int, int]] = None  # (TH, TW) of the tiled paths
    threads: int = 0         # workgroup size cap, multiple of 64
    wg_per_cu: int = 0       # batch kernel: resident workgroups per CU
    max_wgs: int = 0         # batch_run / step_batch: workgroups per launch

    def c(self) -> CParams:
        p = CParams()
        p.L, p.S = int(self.L), int(self.S)
        for i in range(32):
            p.dom[i] = int(self.dom[i]) if i < len(self.dom) else 0
        p.rate_ex, p.rate_sel, p.rate_rep = (float(self.ex), float(self.sel),
                                             float(self.rep))
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.replica = int(self.replica) & 0xFFFFFFFF
        p.flags = FLAG_MOORE if self.moore else 0
        if self.prob is not None:
            P = np.ascontiguousarray(self.prob, dtype=np.float64).reshape(-1)
            if P.size != self.S * self.S:
                raise ValueError("prob must hold S * S entries")
            p.dom_prob = P.ctypes.data
            p._keep = P  # the array must outlive the call
        else:
            p.dom_prob = None
        p.launch.route = ROUTE_CODES[self.route]
        p.launch.tile_h, p.launch.tile_w = (
            (int(self.tile[0]), int(self.tile[1])) if self.tile else (0, 0))
        p.launch.threads = int(self.threads)
        p.launch.wg_per_cu = int(self.wg_per_cu)
        p.launch.max_wgs = int(self.max_wgs)
        return p

    def with_launch(self, **kw) -> "Params":
        """A copy with other launch choices (route, tile, threads,
        wg_per_cu, max_wgs); the job itself is unchanged."""
        return dataclasses.replace(self, **kw)


def circulant_dom(S: int, K) -> list:
    kmask = 0
    for k in K:
        kmask |= 1 << (int(k) % S)
    out = (C.c_uint32 * 32)()
    _check(lib().escg_circulant_dom(S, kmask, out), "escg_circulant_dom")
    return list(out)


def dom_from_matrix(D) -> list:
    D = np.ascontiguousarray(D, dtype=np.uint8)
    S = D.shape[0]
    out = (C.c_uint32 * 32)()
    _check(lib().escg_dom_from_matrix(
        S, D.reshape(-1).ctypes.data_as(C.POINTER(C.c_uint8)), out),
        "escg_dom_from_matrix")
    return list(out)


def thresholds(p: Params):
    t1, t2 = C.c_uint32(), C.c_uint32()
    cp = p.c()
    _check(lib().escg_thresholds(C.byref(cp), C.byref(t1), C.byref(t2)),
           "escg_thresholds")
    return t1.value, t2.value


def eps_from_mobility(M: float, L: int) -> float:
    """Exchange rate for mobility M on an L x L lattice (M = 2 eps / L^2),
    computed by the library."""
    e = C.c_double()
    _check(lib().escg_eps_from_mobility(float(M), int(L), C.byref(e)),
           "escg_eps_from_mobility")
    return e.value


def batch_max_L(S: int = 3) -> int:
    return int(lib().escg_batch_max_L(int(S)))


def tile_plan(p: Params, persistent=True):
    """(TH, TW, threads) the persistent (True), per-MCS (False) or
    multi-job persistent ("multi") tiled path would use for job p with its
    launch choices, or None."""
    a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
    cp = p.c()
    mode = 2 if persistent == "multi" else (1 if persistent else 0)
    s = lib().escg_tile_plan(C.byref(cp), mode,
                             C.byref(a), C.byref(b), C.byref(c))
    if s == EUNSUPPORTED:
        return None
    _check(s, "escg_tile_plan")
    return a.value, b.value, c.value


def last_route() -> str:
    """Path taken by this thread's last step_mcs ("lds", "tiled",
    "persistent")."""
    return ROUTE_NAMES[int(lib().escg_last_route())]


def last_error() -> str:
    return lib().escg_last_error().decode()


def async_status(reset: bool = True) -> None:
    """Raises EscgError if an asynchronous kernel recorded a device error."""
    _check(lib().escg_async_status(1 if reset else 0), "escg_async_status")


# ---------------------------------------------------------------------------
# Device calls (torch tensors)
# ---------------------------------------------------------------------------

def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t, dtype_name: str, numel: Optional[int] = None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if str(t.dtype) != dtype_name:
        raise ValueError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, need {numel}")
    return C.c_void_p(t.data_ptr())


def init(p: Params, lattice, stream=None) -> None:
    cp = p.c()
    _check(lib().escg_init(C.byref(cp), _ptr(lattice, "torch.uint8",
                                             p.L * p.L), _stream(stream)),
           "escg_init")


def densities(p: Params, lattice, counts, stream=None) -> None:
    cp = p.c()
    _check(lib().escg_densities(
        C.byref(cp), _ptr(lattice, "torch.uint8", p.L * p.L),
        _ptr(counts, "torch.int32", p.S + 1), _stream(stream)),
        "escg_densities")


def step_mcs(p: Params, lattice, mcs0: int, n_mcs: int, counts=None,
             stream=None) -> None:
    cp = p.c()
    cptr = (_ptr(counts, "torch.int32", (n_mcs + 1) * (p.S + 1))
            if counts is not None else None)
    _check(lib().escg_step_mcs(C.byref(cp),
                               _ptr(lattice, "torch.uint8", p.L * p.L),
                               int(mcs0), int(n_mcs), cptr, _stream(stream)),
           "escg_step_mcs")


def step_mcs_static(p: Params, lattice, mcs0: int, n_mcs: int, counts=None,
                    stream=None) -> None:
    """step_mcs without any device allocation (escg_step_mcs_static): scratch
    comes from the library's fixed per-GPU array; calls whose work overlaps
    on one GPU must not be issued."""
    cp = p.c()
    cptr = (_ptr(counts, "torch.int32", (n_mcs + 1) * (p.S + 1))
            if counts is not None else None)
    _check(lib().escg_step_mcs_static(
        C.byref(cp), _ptr(lattice, "torch.uint8", p.L * p.L), int(mcs0),
        int(n_mcs), cptr, _stream(stream)), "escg_step_mcs_static")


def run_until_extinction(p: Params, lattice, mcs0: int, max_mcs: int,
                         mode: int, result, stream=None) -> None:
    cp = p.c()
    _check(lib().escg_run_until_extinction(
        C.byref(cp), _ptr(lattice, "torch.uint8", p.L * p.L), int(mcs0),
        int(max_mcs), int(mode), _ptr(result, "torch.int32", p.S + 3),
        _stream(stream)), "escg_run_until_extinction")


def batch_run(params: Sequence[Params], offsets, lattices, max_mcs,
              mode: int, init_lattices: bool, results, mcs0=None,
              stream=None) -> None:
    """``offsets`` / ``max_mcs`` / ``mcs0``: host sequences of length n;
    ``lattices``: one uint8 device tensor holding all lattices; ``results``:
    int32 device tensor of n * 34 words."""
    n = len(params)
    arr = (CParams * max(n, 1))()
    keep = [p.c() for p in params]  # holds any probability arrays
    for i, cp in enumerate(keep):
        arr[i] = cp
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    mx = np.ascontiguousarray(max_mcs, dtype=np.uint32)
    m0 = (np.ascontiguousarray(mcs0, dtype=np.uint32)
          if mcs0 is not None else None)
    assert off.size == n and mx.size == n and (m0 is None or m0.size == n)
    end = max((int(o) + int(q.L) * int(q.L) for o, q in zip(off, params)),
              default=0)
    if lattices.numel() < end:
        raise ValueError("lattice buffer too small for the given offsets")
    _check(lib().escg_batch_run(
        n, arr, off.ctypes.data_as(C.POINTER(C.c_uint64)),
        _ptr(lattices, "torch.uint8"),
        m0.ctypes.data_as(C.POINTER(C.c_uint32)) if m0 is not None else None,
        mx.ctypes.data_as(C.POINTER(C.c_uint32)), int(mode),
        1 if init_lattices else 0,
        _ptr(results, "torch.int32", n * BATCH_RESULT_WORDS),
        _stream(stream)), "escg_batch_run")


def step_batch(params: Sequence[Params], lattices, mcs0, n_mcs,
               stream=None) -> None:
    """Advances each job i (``lattices[i]``: its uint8 device tensor of
    L*L sites) by ``n_mcs[i]`` MCS from MCS ``mcs0[i]``, all jobs together:
    persistent launches holding several jobs, or one launch per MCS when the
    first job's route is "tiled".  Every L must be a multiple of 8
    (>= 16)."""
    n = len(params)
    assert len(lattices) == n and len(mcs0) == n and len(n_mcs) == n
    arr = (CParams * max(n, 1))()
    ptrs = (C.c_void_p * max(n, 1))()
    keep = [p.c() for p in params]  # holds any probability arrays
    for i, (cp, p, t) in enumerate(zip(keep, params, lattices)):
        arr[i] = cp
        ptrs[i] = _ptr(t, "torch.uint8", p.L * p.L).value
    m0 = np.ascontiguousarray(mcs0, dtype=np.uint32)
    nm = np.ascontiguousarray(n_mcs, dtype=np.uint32)
    _check(lib().escg_step_batch(
        n, arr, ptrs, m0.ctypes.data_as(C.POINTER(C.c_uint32)),
        nm.ctypes.data_as(C.POINTER(C.c_uint32)), _stream(stream)),
        "escg_step_batch")
