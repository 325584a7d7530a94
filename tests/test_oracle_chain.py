"""Exact-distribution pins of O1 (random-sequential update) and O2 (2x2-block
schedule) on tiny lattices.

The exact distributions are built here by brute-force enumeration from the
paper's description of one elementary step (Sec. "Single Threaded ESCG in
C++": a uniform cell, a uniform one of its four von Neumann neighbours under
periodic wrap, an action with probabilities proportional to the rates, then
the action's prose semantics).  The oracles are sampled with independent
streams (replica ids) and compared by a G-test.

* L = 2: every site's left and right (and up and down) neighbour coincide,
  the lattice has exactly four edges, each chosen with probability 1/4 and a
  uniform orientation.  One O2 pass uses one 2x2 block that covers the
  lattice and picks one of the same four edges, so one O2 MCS (four passes)
  has the law of four RSU steps.
* L = 3: the RSU chain on 4^9 states with distinct up/down/left/right.
* L = 4: one O2 pass is a uniform mixture over the four block offsets of
  independent per-block updates.
* The same three pins for the 8-way Moore neighbourhood (the paper's
  --neighbourhood 8), whose random-sequential step picks one of eight
  neighbours.
* Probabilistic dominance: the L = 2 chains and the L = 4 one-pass law with
  win probabilities on a mutual matrix, and the exact reductions P = D
  (deterministic) and P = 0 (no selection).
"""
import itertools

import numpy as np
import pytest
from scipy.stats import chi2

import oracle as O
from tests.test_oracle_rule import _prose_rule


def g_test(observed: dict, expected_p: dict, n: int, min_e: float = 5.0):
    """G-test p-value of observed counts against exact probabilities, with
    categories of small expectation pooled into one."""
    keys = set(expected_p) | set(observed)
    for k in observed:
        assert expected_p.get(k, 0.0) > 0.0, f"impossible outcome {k}"
    big = [k for k in keys if expected_p.get(k, 0.0) * n >= min_e]
    small = [k for k in keys if k not in set(big)]
    obs = [observed.get(k, 0) for k in big]
    exp = [expected_p[k] * n for k in big]
    if small:
        obs.append(sum(observed.get(k, 0) for k in small))
        exp.append(sum(expected_p.get(k, 0.0) for k in small) * n)
    obs = np.array(obs, float)
    exp = np.array(exp, float)
    m = obs > 0
    G = 2.0 * np.sum(obs[m] * np.log(obs[m] / exp[m]))
    df = max(len(obs) - 1, 1)
    return chi2.sf(G, df)


def neighbours(r, c, L, nbhd):
    """The 4 von Neumann or 8 Moore neighbours of (r, c) under wrap (with
    repeats on tiny lattices, as a uniform choice of direction gives)."""
    d = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if nbhd == 8:
        d += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    return [((r + dr) % L, (c + dc) % L) for dr, dc in d]


def outcomes(a, x, y, D, P):
    """[(x', y'), prob] of one action on the pair (selected x, neighbour y):
    the prose rule, except that with dominance probabilities P a selection
    tries the selected cell's win first (probability P[x][y] where x
    dominates y) and then the neighbour's (P[y][x] where y dominates x)."""
    if P is None or a != O.SELECTION or x == y or x == 0 or y == 0:
        return [(_prose_rule(a, x, y, D), 1.0)]
    pxy = P[x - 1, y - 1] if D[x - 1, y - 1] else 0.0
    pyx = P[y - 1, x - 1] if D[y - 1, x - 1] else 0.0
    return [((x, 0), pxy), ((0, y), (1 - pxy) * pyx),
            ((x, y), (1 - pxy) * (1 - pyx))]


def rsu_step_dist(L, S, D, rates, dist, nbhd=4, P=None):
    """One random-sequential step applied to a distribution over lattices
    (dict tuple -> prob): a uniform cell, a uniform one of its nbhd
    neighbours (direction chosen uniformly, wrap), an action by rate."""
    ex, sel, rep = rates
    tot = ex + sel + rep
    pa = {O.EXCHANGE: ex / tot, O.SELECTION: sel / tot,
          O.REPRODUCTION: rep / tot}
    N = L * L
    out = {}
    for state, p in dist.items():
        for i in range(N):
            r, c = divmod(i, L)
            for nr, nc in neighbours(r, c, L, nbhd):
                j = nr * L + nc
                for a, q in pa.items():
                    if q == 0.0:
                        continue
                    for (xn, yn), qo in outcomes(a, state[i], state[j], D, P):
                        s = list(state)
                        s[i], s[j] = xn, yn
                        t = tuple(s)
                        out[t] = out.get(t, 0.0) + p * q * qo / (nbhd * N)
    return out


def sample(fn, n):
    hist = {}
    for rep in range(n):
        t = tuple(int(v) for v in fn(rep))
        hist[t] = hist.get(t, 0) + 1
    return hist


RATES = [(1.0, 1.0, 2.0), (0.5, 1.0, 1.0)]
# An imported, non-antisymmetric matrix (1 and 2 beat each other, 3 beats 1):
# here the orientation of the chosen pair matters.
D_MUTUAL = np.array([[0, 1, 0], [1, 0, 0], [1, 0, 0]], np.uint8)


@pytest.mark.parametrize("rates", RATES)
@pytest.mark.parametrize("mutual", [False, True])
def test_L2_rsu_matches_exact_chain(rates, mutual):
    L, S = 2, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    g0 = np.array([1, 2, 0, 3], np.uint8)
    steps = 4
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(steps):
        dist = rsu_step_dist(L, S, D, rates, dist)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=11, replica=rep)
        g = g0.copy()
        O.o1_steps(job, g, 0, steps)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("rates", RATES)
@pytest.mark.parametrize("mutual", [False, True])
def test_L2_block_schedule_mcs_equals_four_rsu_steps(rates, mutual):
    L, S = 2, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    g0 = np.array([3, 0, 2, 1], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(8):
        dist = rsu_step_dist(L, S, D, rates, dist)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=5, replica=rep)
        g = g0.copy()
        O.o2_run(job, g, 17, 2, want_counts=False)  # two MCS = 8 passes
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("mutual", [False, True])
def test_L3_rsu_matches_exact_chain(mutual):
    # with the mutual pair (2 over 1 in column 1) the orientation of a
    # vertical pair matters, so "up" and "down" are told apart
    L, S = 3, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 3, 0, 1, 2, 3, 0, 2], np.uint8)
    steps = 3
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(steps):
        dist = rsu_step_dist(L, S, D, rates, dist)
    n = 30000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=3, replica=rep)
        g = g0.copy()
        O.o1_steps(job, g, 1000, steps)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


def block_pass_dist(L, S, D, rates, g0, nbhd=4, P=None):
    """Exact law of one O2 pass from g0: offsets uniform on {0,1}^2; the
    (L/2)^2 disjoint 2x2 blocks update independently, each on one of its
    internal pairs with a uniform orientation and an action drawn with
    probability proportional to the rates.  Von Neumann: the 4 edges, each
    1/4.  Moore: the 4 edges 1/8 each and the 2 diagonals 1/4 each (a
    diagonal lies in a block for one offset in four, an edge for one in
    two, so these weights give every Moore pair the same rate)."""
    ex, sel, rep = rates
    tot = ex + sel + rep
    pa = [(O.EXCHANGE, ex / tot), (O.SELECTION, sel / tot),
          (O.REPRODUCTION, rep / tot)]
    total = {}
    for ox, oy in itertools.product((0, 1), repeat=2):
        per_block = []
        for by, bx in itertools.product(range(L // 2), repeat=2):
            r0, c0 = 2 * by + oy, 2 * bx + ox
            r1, c1 = (r0 + 1) % L, (c0 + 1) % L
            A, B, C_, Dd = (r0 * L + c0, r0 * L + c1, r1 * L + c0,
                            r1 * L + c1)
            sites = (A, B, C_, Dd)
            res = {}
            pairs = [((A, B), 1), ((C_, Dd), 1), ((A, C_), 1), ((B, Dd), 1)]
            if nbhd == 8:
                pairs += [((A, Dd), 2), ((B, C_), 2)]
            wsum = sum(wt for _, wt in pairs)
            for (f, s), wt in pairs:
                for cell, nbr in ((f, s), (s, f)):
                    for a, q in pa:
                        for (xn, yn), qo in outcomes(a, int(g0[cell]),
                                                     int(g0[nbr]), D, P):
                            loc = {k: int(g0[k]) for k in sites}
                            loc[cell], loc[nbr] = xn, yn
                            key = tuple(loc[k] for k in sites)
                            res[key] = (res.get(key, 0.0) +
                                        q * qo * wt / (2 * wsum))
            per_block.append((sites, res))
        joint = {tuple(g0.tolist()): 1.0}
        for sites, res in per_block:
            nxt = {}
            for st, p in joint.items():
                for vals, q in res.items():
                    s = list(st)
                    for k, v in zip(sites, vals):
                        s[k] = v
                    t = tuple(s)
                    nxt[t] = nxt.get(t, 0.0) + p * q
            joint = nxt
        for st, p in joint.items():
            total[st] = total.get(st, 0.0) + p / 4
    return total


@pytest.mark.parametrize("mutual", [False, True])
def test_L4_one_pass_matches_exact_block_law(mutual):
    L, S = 4, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 0, 3,
                   3, 3, 1, 0,
                   0, 2, 2, 1,
                   1, 0, 3, 2], np.uint8)
    dist = block_pass_dist(L, S, D, rates, g0)
    assert abs(sum(dist.values()) - 1.0) < 1e-9
    n = 40000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=9, replica=rep)
        g = g0.copy()
        O.o2_pass(job, g, 3, rep % 4)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


# --- Moore (8-way) neighbourhood ------------------------------------------
# On L = 2 a site's eight Moore neighbours are its row neighbour twice, its
# column neighbour twice and its diagonal neighbour four times, so a
# random-sequential step picks each axis edge with probability 1/8 and each
# diagonal with 1/4: exactly the slot weights of one 2x2 block.  One O2 MCS
# therefore has the law of four RSU steps here too.


@pytest.mark.parametrize("mutual", [False, True])
def test_L2_moore_rsu_matches_exact_chain(mutual):
    L, S = 2, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 0, 3], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(4):
        dist = rsu_step_dist(L, S, D, rates, dist, nbhd=8)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=13, replica=rep, nbhd=8)
        g = g0.copy()
        O.o1_steps(job, g, 0, 4)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("rates", RATES)
@pytest.mark.parametrize("mutual", [False, True])
def test_L2_moore_block_schedule_mcs_equals_four_rsu_steps(rates, mutual):
    L, S = 2, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    g0 = np.array([3, 0, 2, 1], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(8):
        dist = rsu_step_dist(L, S, D, rates, dist, nbhd=8)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=6, replica=rep, nbhd=8)
        g = g0.copy()
        O.o2_run(job, g, 4, 2, want_counts=False)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("mutual", [False, True])
def test_L3_moore_rsu_matches_exact_chain(mutual):
    # eight distinct neighbours on L = 3
    L, S = 3, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 3, 0, 1, 2, 3, 0, 2], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(3):
        dist = rsu_step_dist(L, S, D, rates, dist, nbhd=8)
    n = 30000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=4, replica=rep, nbhd=8)
        g = g0.copy()
        O.o1_steps(job, g, 500, 3)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("mutual", [False, True])
def test_L4_moore_one_pass_matches_exact_block_law(mutual):
    L, S = 4, 3
    D = D_MUTUAL if mutual else O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 0, 3,
                   3, 3, 1, 0,
                   0, 2, 2, 1,
                   1, 0, 3, 2], np.uint8)
    dist = block_pass_dist(L, S, D, rates, g0, nbhd=8)
    assert abs(sum(dist.values()) - 1.0) < 1e-9
    n = 40000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=10, replica=rep, nbhd=8)
        g = g0.copy()
        O.o2_pass(job, g, 3, rep % 4)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


def test_moore_law_differs_from_von_neumann():
    # the Moore pins are not the von Neumann ones under another name: the
    # exact one-pass laws differ, and Moore samples reject the 4-way law
    L, S = 4, 3
    D = O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 0, 3, 3, 3, 1, 0, 0, 2, 2, 1, 1, 0, 3, 2], np.uint8)
    vn = block_pass_dist(L, S, D, rates, g0, nbhd=4)
    n = 40000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=10, replica=rep, nbhd=8)
        g = g0.copy()
        O.o2_pass(job, g, 3, rep % 4)
        return g
    obs = sample(run, n)
    vn = {k: vn.get(k, 0.0) + 1e-12 for k in set(vn) | set(obs)}
    assert g_test(obs, vn, n) < 1e-6


# --- Probabilistic dominance -----------------------------------------------
# Dominance probabilities on a mutual matrix (1 and 2 beat each other, 3
# beats 1), so both orders of the two win tests matter.
P_MUTUAL = np.array([[0.0, 0.35, 0.0], [0.6, 0.0, 0.0], [0.25, 0.0, 0.0]])


@pytest.mark.parametrize("nbhd", [4, 8])
def test_L2_probabilistic_rsu_matches_exact_chain(nbhd):
    L, S = 2, 3
    rates = (0.5, 2.0, 1.0)
    g0 = np.array([1, 2, 0, 3], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(4):
        dist = rsu_step_dist(L, S, D_MUTUAL, rates, dist, nbhd=nbhd,
                             P=P_MUTUAL)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D_MUTUAL, *rates, seed=21, replica=rep, nbhd=nbhd,
                    P=P_MUTUAL)
        g = g0.copy()
        O.o1_steps(job, g, 0, 4)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("nbhd", [4, 8])
def test_L2_probabilistic_block_schedule_mcs_equals_four_rsu_steps(nbhd):
    # O2 quantises each probability to multiples of 1 / (T2 - T1) ~ 2^-23:
    # far below what 20000 samples resolve
    L, S = 2, 3
    rates = (0.5, 2.0, 1.0)
    g0 = np.array([3, 1, 2, 1], np.uint8)
    dist = {tuple(g0.tolist()): 1.0}
    for _ in range(4):
        dist = rsu_step_dist(L, S, D_MUTUAL, rates, dist, nbhd=nbhd,
                             P=P_MUTUAL)
    n = 20000

    def run(rep):
        job = O.Job(L, S, D_MUTUAL, *rates, seed=8, replica=rep, nbhd=nbhd,
                    P=P_MUTUAL)
        g = g0.copy()
        O.o2_run(job, g, 2, 1, want_counts=False)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


def test_L4_probabilistic_one_pass_matches_exact_block_law():
    L, S = 4, 3
    rates = (0.5, 2.0, 1.0)
    g0 = np.array([1, 2, 0, 3, 3, 3, 1, 0, 0, 2, 2, 1, 1, 0, 3, 2], np.uint8)
    dist = block_pass_dist(L, S, D_MUTUAL, rates, g0, P=P_MUTUAL)
    assert abs(sum(dist.values()) - 1.0) < 1e-9
    n = 40000

    def run(rep):
        job = O.Job(L, S, D_MUTUAL, *rates, seed=12, replica=rep, P=P_MUTUAL)
        g = g0.copy()
        O.o2_pass(job, g, 3, rep % 4)
        return g
    assert g_test(sample(run, n), dist, n) > 1e-4


@pytest.mark.parametrize("runner", ["o1", "o2"])
@pytest.mark.parametrize("nbhd", [4, 8])
def test_probabilities_equal_to_the_matrix_give_the_deterministic_rule(
        runner, nbhd):
    # P = D: every permitted win succeeds, the rule is the deterministic
    # one, run for run; P = 0 removes all selection, as D = 0 does
    L, S = 12, 5
    D = O.circulant_matrix(S, [1, 3])
    D[0, 1] = 0
    run = O.o1_run if runner == "o1" else O.o2_run
    g0 = np.random.default_rng(3).integers(0, S + 1, L * L, dtype=np.uint8)
    for P, Dref in ((D.astype(np.float64), D),
                    (np.zeros((S, S)), np.zeros((S, S), np.uint8))):
        a, b = g0.copy(), g0.copy()
        ca = run(O.Job(L, S, D, 0.7, 1.3, 1.0, seed=4, nbhd=nbhd, P=P), a,
                 3, 6)
        cb = run(O.Job(L, S, Dref, 0.7, 1.3, 1.0, seed=4, nbhd=nbhd), b, 3, 6)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)


def test_g_test_detects_a_planted_rule_error():
    # Sanity of the harness itself: the exact L=2 law with reproduction
    # swapped for a no-op must be rejected against real O1 samples.
    L, S = 2, 3
    D = O.circulant_matrix(S, [1])
    rates = (1.0, 1.0, 2.0)
    g0 = np.array([1, 2, 0, 3], np.uint8)
    wrong = {tuple(g0.tolist()): 1.0}
    for _ in range(4):
        wrong = rsu_step_dist(L, S, D, (1.0, 1.0, 0.0), wrong)
    n = 5000

    def run(rep):
        job = O.Job(L, S, D, *rates, seed=11, replica=rep)
        g = g0.copy()
        O.o1_steps(job, g, 0, 4)
        return g
    obs = sample(run, n)
    wrong = {k: wrong.get(k, 0.0) + 1e-12 for k in set(wrong) | set(obs)}
    assert g_test(obs, wrong, n) < 1e-6
