"""Pins of the oracle's per-pair arithmetic: the pair rule, the dominance
matrix, the action thresholds and the initial-lattice map, each against what
the paper (or plain mathematics) fixes independently of the oracle's code."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

G = os.path.join(os.path.dirname(__file__), "golden")

# Numeric labels for RPS such that C(3, {1}) ("i beats i+1") is the usual game
# (rock blunts scissors, scissors cut paper, paper wraps rock).
RPS_LABEL = {"_": 0, "R": 1, "S": 2, "P": 3}
ACTION = {"eps": O.EXCHANGE, "mu": O.SELECTION, "sigma": O.REPRODUCTION}


def _rows(name):
    with open(os.path.join(G, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("row", _rows("rps_transitions.txt"))
def test_paper_worked_transitions(row):
    act, x, y, x2, y2 = row
    D = O.circulant_matrix(3, [1])
    got = O.pair_rule(ACTION[act], RPS_LABEL[x], RPS_LABEL[y], D)
    assert got == (RPS_LABEL[x2], RPS_LABEL[y2])


def test_rpsls_matrix_matches_paper_figure():
    # The figure's edge list, labelled so that C(5, {1, 2}) applies.
    lab = {"Rock": 1, "Scissors": 2, "Lizard": 3, "Paper": 4, "Spock": 5}
    fig = np.zeros((5, 5), np.uint8)
    for a, b in _rows("rpsls_figure_edges.txt"):
        fig[lab[a] - 1, lab[b] - 1] = 1
    assert np.array_equal(O.circulant_matrix(5, [1, 2]), fig)
    # Every species beats exactly two others and loses to two (a tournament).
    assert (fig.sum(0) == 2).all() and (fig.sum(1) == 2).all()
    assert not (fig & fig.T).any()


def test_circulant_rps_and_i_beats_i1_i3():
    D3 = O.circulant_matrix(3, [1])
    assert D3.tolist() == [[0, 1, 0], [0, 0, 1], [1, 0, 0]]
    D5 = O.circulant_matrix(5, [1, 3])
    for i in range(1, 6):
        for j in range(1, 6):
            beats = j == (i % 5) + 1 or j == ((i + 2) % 5) + 1
            assert D5[i - 1, j - 1] == int(beats), (i, j)


def _prose_rule(action, x, y, D):
    """The three actions as the paper's bullet list states them (Sec.
    "Single Threaded ESCG in C++"): interaction empties the losing site of
    two occupied different species; reproduction fills the empty one of the
    two sites with the other's species; migration swaps the two sites.
    Identical species never change."""
    if x == y:
        return x, y
    if action == O.EXCHANGE:
        return y, x
    if action == O.SELECTION:
        if x == 0 or y == 0:
            return x, y
        if D[x - 1, y - 1]:
            return x, 0
        if D[y - 1, x - 1]:
            return 0, y
        return x, y
    if (x == 0) != (y == 0):
        s = x | y
        return s, s
    return x, y


@pytest.mark.parametrize("S,K", [(3, [1]), (5, [1, 3]), (5, [1, 2]), (4, [1]),
                                 (2, [1]), (1, [])])
def test_pair_rule_truth_table(S, K):
    D = O.circulant_matrix(S, K) if K else np.zeros((S, S), np.uint8)
    for a, x, y in itertools.product(range(3), range(S + 1), range(S + 1)):
        assert O.pair_rule(a, x, y, D) == _prose_rule(a, x, y, D), (a, x, y)


def test_pair_rule_mutual_dominance_selected_cell_wins():
    # An imported matrix may let two species beat each other; the paper's
    # rule tests the selected cell first, so the neighbour is emptied.
    D = np.array([[0, 1], [1, 0]], np.uint8)
    assert O.pair_rule(O.SELECTION, 1, 2, D) == (1, 0)
    assert O.pair_rule(O.SELECTION, 2, 1, D) == (2, 0)


@pytest.mark.parametrize("rates", [(0.5, 1, 1), (1, 1, 1), (13.1072, 1, 1),
                                   (51.2, 1, 1), (0.002, 1, 1), (1280, 1, 1),
                                   (0, 1, 1), (1, 0, 1), (1, 1, 0), (0, 0, 1),
                                   (1e-9, 1, 1), (3, 2, 5)])
def test_thresholds_are_floor_of_exact_probabilities(rates):
    ex, sel, rep = rates
    T1, T2 = O.thresholds(ex, sel, rep)
    fe, fs, fr = (Fraction(v) for v in rates)
    tot = fe + fs + fr
    e1 = (fe / tot) * 2**24
    e2 = ((fe + fs) / tot) * 2**24
    # floor of the exact value, except where double rounding of the ratio
    # lands exactly on an integer boundary (off by at most one step).
    assert abs(T1 - int(e1)) <= 1 and abs(T2 - int(e2)) <= 1
    assert 0 <= T1 <= T2 <= 2**24
    assert abs(Fraction(T1, 2**24) - fe / tot) <= Fraction(1, 2**23)
    if rep == 0:
        assert T2 == 2**24
    if ex == 0:
        assert T1 == 0


@pytest.mark.parametrize("S", [1, 3, 5, 8])
def test_init_is_uniform_over_species_and_empty(S):
    from scipy.stats import chisquare
    L = 256
    g = O.init_lattice(L, S, seed=7, replica=3)
    assert g.max() <= S
    c = np.bincount(g, minlength=S + 1)
    assert c.sum() == L * L
    assert chisquare(c).pvalue > 1e-4
    # different replica ids give different (independent) lattices
    g2 = O.init_lattice(L, S, seed=7, replica=4)
    assert (g != g2).mean() > 0.5 * S / (S + 1)


def test_init_map_is_floor_scaling():
    # site n takes word n&3 of one Philox call per four sites
    S, seed, rep = 5, 0x1234_5678_9ABC, 2
    g = O.init_lattice(4, S, seed, rep)
    for n in range(16):
        w = O.philox4x32([n >> 2, 0, 1 << 8, rep],
                         [seed & 0xFFFFFFFF, seed >> 32],
                         O.SCHEDULE_ROUNDS)[n & 3]
        assert g[n] == (int(w) * (S + 1)) >> 32
