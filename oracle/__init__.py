"""CPU oracle for the ESCG Monte Carlo hot path (arxiv 2508.16639).

TEST INFRASTRUCTURE ONLY.  The product package never imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may.  The arithmetic lives in ``escg_oracle.c`` (plain C, one
thread); this file only compiles it with gcc and marshals arguments.

O1 is the paper's random-sequential update (Algorithm "Elementary Step"
inside Algorithm "Overall ESCG Loop"); O2 is the parallel 2x2-block schedule
whose exact result the GPU path must reproduce byte for byte.  See the C file
for the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ESCG_ORACLE_SRC names another copy of the C source to build and load
# instead (the mutation tests plant mistakes in such a copy, never here).
_SRC = os.environ.get("ESCG_ORACLE_SRC") or os.path.join(_HERE,
                                                         "escg_oracle.c")
_OUT_DIR = (os.path.join(os.path.dirname(os.path.abspath(_SRC)), "_build")
            if os.environ.get("ESCG_ORACLE_SRC") else
            os.path.join(_HERE, "_build"))
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")

# Rounds of the Philox4x32 generator the block schedule (O2) and the init
# draw from: 7, the fewest with which Salmon et al. (SC'11) report
# Philox4x32 passing TestU01's BigCrush.  The paper uses Mersenne Twister and
# cuRAND, so the generator is a parameter of this schedule, not the paper's.
SCHEDULE_ROUNDS = 7

FIRST_EXTINCTION = 0
MONOCULTURE = 1
EXCHANGE, SELECTION, REPRODUCTION = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math: the thresholds are
    IEEE double)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u32 = C.c_uint32
        dbl = C.c_double
        job = [u32, u32, u8p, dbl, dbl, dbl, C.c_uint64, u32, C.c_int,
               C.c_int, C.c_void_p]
        L.orc_philox4x32.argtypes = [u32p, u32p, C.c_int, u32p]
        L.orc_circulant_matrix.argtypes = [u32, u32, u8p]
        L.orc_pair_rule.argtypes = [C.c_int, C.c_uint8, C.c_uint8, u32, u8p,
                                    u8p]
        L.orc_thresholds.argtypes = [dbl, dbl, dbl, C.POINTER(u32),
                                     C.POINTER(u32)]
        L.orc_init.argtypes = [u32, u32, C.c_uint64, u32, C.c_int, u8p]
        L.orc_counts.argtypes = [u32, u32, u8p, u32p]
        L.orc_o2_pass.argtypes = job + [u32, u32, u8p]
        L.orc_o2_run.argtypes = job + [u32, u32, u8p, C.c_void_p]
        L.orc_o2_run_until.argtypes = job + [u32, u32, C.c_int, u8p, u32p]
        L.orc_o1_run.argtypes = job + [u32, u32, u8p, C.c_void_p]
        L.orc_o1_steps.argtypes = job + [C.c_uint64, C.c_uint64, u8p]
        L.orc_o1_run_until.argtypes = job + [u32, u32, C.c_int, u8p, u32p]
        for f in (L.orc_philox4x32, L.orc_circulant_matrix, L.orc_pair_rule,
                  L.orc_thresholds, L.orc_init, L.orc_counts, L.orc_o2_pass,
                  L.orc_o2_run, L.orc_o2_run_until, L.orc_o1_run,
                  L.orc_o1_steps, L.orc_o1_run_until):
            f.restype = None
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Primitive wrappers
# ---------------------------------------------------------------------------

def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32(c, k, rounds, out)
    return out


def circulant_matrix(S: int, K) -> np.ndarray:
    """Flat S*S uint8 dominance matrix of the circulant graph C(S, K)."""
    kmask = 0
    for k in K:
        kmask |= 1 << (int(k) % S)
    D = np.zeros(S * S, np.uint8)
    lib().orc_circulant_matrix(S, kmask, D)
    return D.reshape(S, S)


def pair_rule(action: int, x: int, y: int, D: np.ndarray):
    D = np.ascontiguousarray(D, dtype=np.uint8)
    out = np.zeros(2, np.uint8)
    lib().orc_pair_rule(action, x, y, D.shape[0], D.reshape(-1), out)
    return int(out[0]), int(out[1])


def thresholds(ex: float, sel: float, rep: float):
    t1, t2 = C.c_uint32(), C.c_uint32()
    lib().orc_thresholds(ex, sel, rep, C.byref(t1), C.byref(t2))
    return t1.value, t2.value


def init_lattice(L: int, S: int, seed: int, replica: int = 0,
                 rounds: int = SCHEDULE_ROUNDS) -> np.ndarray:
    g = np.zeros(L * L, np.uint8)
    lib().orc_init(L, S, seed, replica, rounds, g)
    return g


def counts(grid: np.ndarray, L: int, S: int) -> np.ndarray:
    c = np.zeros(S + 1, np.uint32)
    lib().orc_counts(L, S, np.ascontiguousarray(grid, np.uint8), c)
    return c


# ---------------------------------------------------------------------------
# Jobs
# ---------------------------------------------------------------------------

@dataclass
class Job:
    """One simulation: lattice side L (even for O2), S species with flat
    dominance matrix D (S x S, paper layout), rates by role (exchange =
    migration, selection = interaction, reproduction), the RNG key, and the
    neighbourhood (4-way von Neumann or 8-way Moore, the paper's
    --neighbourhood option) and optional dominance probabilities P (entry
    (a-1, b-1): probability that a selection of a against b succeeds, used
    where D says a dominates b; None = deterministic)."""
    L: int
    S: int
    D: np.ndarray
    ex: float
    sel: float = 1.0
    rep: float = 1.0
    seed: int = 1
    replica: int = 0
    rounds: int = SCHEDULE_ROUNDS
    nbhd: int = 4          # 4: von Neumann, 8: Moore
    P: Optional[np.ndarray] = None  # S x S dominance probabilities or None
    _Dflat: np.ndarray = field(init=False, repr=False)
    _Pflat: Optional[np.ndarray] = field(init=False, repr=False)

    def __post_init__(self):
        D = np.ascontiguousarray(self.D, dtype=np.uint8).reshape(-1)
        assert D.size == self.S * self.S
        assert self.nbhd in (4, 8)
        self._Pflat = None
        if self.P is not None:
            P = np.ascontiguousarray(self.P, dtype=np.float64).reshape(-1)
            assert P.size == self.S * self.S
            assert ((P >= 0.0) & (P <= 1.0)).all()
            self._Pflat = P
        self._Dflat = D

    def args(self):
        return (self.L, self.S, self._Dflat, float(self.ex), float(self.sel),
                float(self.rep), int(self.seed), int(self.replica),
                int(self.rounds), int(self.nbhd),
                None if self._Pflat is None else self._Pflat.ctypes.data)

    def init(self) -> np.ndarray:
        return init_lattice(self.L, self.S, self.seed, self.replica,
                            self.rounds)


def _grid(grid, L):
    assert grid.dtype == np.uint8 and grid.flags.c_contiguous
    assert grid.size == L * L
    return grid


def o2_pass(job: Job, grid: np.ndarray, t: int, p: int) -> None:
    lib().orc_o2_pass(*job.args(), t, p, _grid(grid, job.L))


def o2_run(job: Job, grid: np.ndarray, mcs0: int, n_mcs: int,
           want_counts: bool = True):
    """Advances `grid` in place by n_mcs MCS; returns counts[(n_mcs+1), S+1]
    or None."""
    assert job.L % 2 == 0
    c = np.zeros((n_mcs + 1, job.S + 1), np.uint32) if want_counts else None
    lib().orc_o2_run(*job.args(), mcs0, n_mcs, _grid(grid, job.L),
                     c.ctypes.data if c is not None else None)
    return c


def o2_run_until(job: Job, grid: np.ndarray, mcs0: int, max_mcs: int,
                 mode: int = FIRST_EXTINCTION) -> np.ndarray:
    """Returns {flag, t_ext, counts[0..S]} as uint32[S+3]."""
    assert job.L % 2 == 0
    r = np.zeros(job.S + 3, np.uint32)
    lib().orc_o2_run_until(*job.args(), mcs0, max_mcs, mode,
                           _grid(grid, job.L), r)
    return r


def o1_run(job: Job, grid: np.ndarray, mcs0: int, n_mcs: int,
           want_counts: bool = True):
    c = np.zeros((n_mcs + 1, job.S + 1), np.uint32) if want_counts else None
    lib().orc_o1_run(*job.args(), mcs0, n_mcs, _grid(grid, job.L),
                     c.ctypes.data if c is not None else None)
    return c


def o1_steps(job: Job, grid: np.ndarray, k0: int, n: int) -> None:
    lib().orc_o1_steps(*job.args(), k0, n, _grid(grid, job.L))


def o1_run_until(job: Job, grid: np.ndarray, mcs0: int, max_mcs: int,
                 mode: int = FIRST_EXTINCTION) -> np.ndarray:
    r = np.zeros(job.S + 3, np.uint32)
    lib().orc_o1_run_until(*job.args(), mcs0, max_mcs, mode,
                           _grid(grid, job.L), r)
    return r
