"""Seeded synthetic workloads for the ESCG hot path.

This module only describes inputs: lattice sizes, species counts and
dominance offsets, rates, seeds, replica tables and request streams.  It holds
none of the method's arithmetic and imports nothing from the rest of the
package, so tests, the oracle side and the benchmark can all use it.

Conventions
-----------
* Rates are named by role: ``ex`` (exchange, the paper's migration),
  ``sel`` (selection, the paper's interaction) and ``rep`` (reproduction).
* Mobility M is converted to an exchange rate with eps = M * L^2 / 2, i.e.
  M = 2 eps / L^2, the definition the workloads are stated in.  (The paper's
  own text writes eps = 2 M N; the two differ by a factor 4 and the workloads
  below are specified in the former.)
* Dominance is a circulant graph C(S, K): species i beats i + k (mod S) for
  every k in K.  RPS is C(3, {1}); the RPSLS workload here is C(5, {1, 3})
  ("i beats i+1 and i+3"), isomorphic to the paper's C(5, {1, 2}).
* Initial lattices are i.i.d. uniform over {0, ..., S} (0 = empty) and are
  drawn by the method's own counter-based generator from (seed, replica), so
  a workload is fully described by the numbers below.
"""
from __future__ import annotations

from dataclasses import dataclass, asdict
from typing import List, Tuple

import numpy as np

RPS = (3, (1,))
RPSLS = (5, (1, 3))
RPSLS_PAPER = (5, (1, 2))


def eps_from_mobility(M: float, L: int) -> float:
    """Exchange rate for mobility M on an L x L lattice (M = 2 eps / L^2)."""
    return float(M) * float(L) * float(L) / 2.0


@dataclass(frozen=True)
class Sim:
    """One single-lattice simulation request."""
    name: str
    L: int
    S: int
    K: Tuple[int, ...]
    ex: float
    sel: float
    rep: float
    mcs: int
    seed: int = 1
    replica: int = 0

    def as_dict(self):
        return asdict(self)


# The single-lattice workloads.  RPS at L=64 is the small parity case; RPS at
# L=512 records densities every MCS; RPSLS at L=3200 is the large-lattice
# throughput case (10.24 M sites).
RPS64 = Sim("rps_L64", 64, *RPS, ex=0.5, sel=1.0, rep=1.0, mcs=100, seed=1)
RPS512 = Sim("rps_L512", 512, *RPS, ex=eps_from_mobility(1e-4, 512), sel=1.0,
             rep=1.0, mcs=10_000, seed=1)
RPSLS3200 = Sim("rpsls_L3200", 3200, *RPSLS, ex=eps_from_mobility(1e-5, 3200),
                sel=1.0, rep=1.0, mcs=1_000, seed=1)
SINGLE = {s.name: s for s in (RPS64, RPS512, RPSLS3200)}


@dataclass
class ReplicaTable:
    """Independent RPS replicas for the batched extinction workload."""
    L: np.ndarray        # uint32, lattice side per replica
    M: np.ndarray        # float64 mobility per replica
    ex: np.ndarray       # float64 exchange rate per replica
    max_mcs: np.ndarray  # uint32 MCS cap per replica (20 L)
    seed: int
    S: int = 3
    K: Tuple[int, ...] = (1,)

    def __len__(self):
        return int(self.L.size)


def batch_replicas(n: int = 4096, seed: int = 1,
                   sizes=(64, 128, 192, 256), logM=(-6.0, -3.0),
                   cap_per_L: int = 20) -> ReplicaTable:
    """n RPS replicas; L uniform over `sizes`, log10 M uniform on `logM`,
    stop at first extinction or cap_per_L * L MCS.  Replica r uses key
    `seed` and replica id r."""
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(sizes, dtype=np.uint32), size=n)
    M = 10.0 ** rng.uniform(logM[0], logM[1], size=n)
    ex = M * L.astype(np.float64) ** 2 / 2.0
    cap = (cap_per_L * L).astype(np.uint32)
    return ReplicaTable(L=L.astype(np.uint32), M=M, ex=ex, max_mcs=cap,
                        seed=seed)


@dataclass(frozen=True)
class Request:
    """One job of the serving workload."""
    job_id: int
    arrival_s: float
    L: int
    S: int
    K: Tuple[int, ...]
    M: float
    ex: float
    mcs: int
    seed: int


def serving_requests(n: int = 2000, rate_per_s: float = 200.0, seed: int = 2,
                     sizes=(100, 200, 400, 800, 1600), logM=(-6.0, -3.0),
                     mcs_range=(500, 5000)) -> List[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate); S in {3, 5} with
    probability 1/2 each; L uniform over `sizes`; log10 M uniform on `logM`;
    MCS budget uniform integer on `mcs_range` (inclusive); job seed = job id
    (replica id 0)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        S, K = RPS if rng.random() < 0.5 else RPSLS
        L = int(rng.choice(sizes))
        M = float(10.0 ** rng.uniform(*logM))
        mcs = int(rng.integers(mcs_range[0], mcs_range[1] + 1))
        out.append(Request(job_id=i, arrival_s=float(t[i]), L=L, S=S, K=K,
                           M=M, ex=eps_from_mobility(M, L), mcs=mcs,
                           seed=i + 1))
    return out


def random_lattice(L: int, S: int, seed: int, domain: int = 1) -> np.ndarray:
    """An arbitrary test lattice (uint8[L*L], values 0..S) drawn with numpy,
    independent of the method's generator.  domain > 1 paints uniform
    domain x domain patches, so that many neighbour pairs share a species."""
    rng = np.random.default_rng(seed)
    if domain <= 1:
        return rng.integers(0, S + 1, size=L * L, dtype=np.uint8)
    nb = (L + domain - 1) // domain
    coarse = rng.integers(0, S + 1, size=(nb, nb), dtype=np.uint8)
    g = np.kron(coarse, np.ones((domain, domain), np.uint8))[:L, :L]
    return np.ascontiguousarray(g.reshape(-1))
