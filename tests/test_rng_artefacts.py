"""Random-number artefact screens of the oracle (CPU).

The paper's Metal version drew from per-thread Mersenne Twister streams and
showed vertical stripes until a burn-in was added (Sec. on the Metal
Mersenne Twister).  Here the screen is a fact of the method: with selection
and reproduction off (sigma = mu = 0) every action is an exchange, whose
swap decisions do not look at the species, so the lattice after any number
of MCS is the initial i.i.d. uniform lattice permuted by a permutation drawn
independently of it, and stays i.i.d. uniform over {0..S}.  Equal-neighbour
fractions and per-row / per-column counts must therefore sit at their
i.i.d. values at every time, for the init draw and for the block schedule
(O2) and the random-sequential update (O1) alike.  A generator with
correlated draws between sites, or a schedule whose swaps depended on the
values, fails it.
"""
import numpy as np
import pytest

import oracle as O
from tests.lattice_stats import screen


@pytest.mark.parametrize("S,seed", [(3, 1), (5, 7)])
def test_init_has_no_spatial_correlation(S, seed):
    L = 512
    g = O.init_lattice(L, S, seed, replica=3).reshape(L, L)
    assert screen(g, S + 1) == []


@pytest.mark.parametrize("nbhd", [4, 8])
def test_exchange_only_o2_stays_iid(nbhd):
    L, S = 256, 3
    job = O.Job(L, S, O.circulant_matrix(S, [1]), 5.0, 0.0, 0.0, seed=11,
                replica=2, nbhd=nbhd)
    g = job.init()
    for _ in range(4):
        O.o2_run(job, g, 0, 8, want_counts=False)
        assert screen(g.reshape(L, L), S + 1) == []


def test_exchange_only_o1_stays_iid():
    L, S = 128, 5
    job = O.Job(L, S, O.circulant_matrix(S, [1, 3]), 5.0, 0.0, 0.0, seed=5,
                replica=1)
    g = job.init()
    O.o1_run(job, g, 0, 10, want_counts=False)
    assert screen(g.reshape(L, L), S + 1) == []


def test_screen_detects_correlated_draws():
    """The screen itself: a lattice whose sites repeat in pairs four
    columns apart (the mark of draws shared between sites), and one with
    one column in eight biased (a stripe), both fail."""
    rng = np.random.default_rng(0)
    L, K = 256, 4
    g = rng.integers(0, K, (L, L), dtype=np.uint8)
    h = g.copy()
    h[:, 4::8] = h[:, 0::8]
    assert any("(0,4)" in b for b in screen(h, K))
    s = g.copy()
    col = s[:, ::8]
    col[rng.random(col.shape) < 0.2] = 0
    s[:, ::8] = col
    assert any("columns" in b for b in screen(s, K))
    assert screen(g, K) == []
