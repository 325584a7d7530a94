"""Spatial statistics of a lattice for the random-number artefact screens.

For sites drawn i.i.d. uniform over K values, the indicators [x_i = x_j] of
distinct pairs at a fixed displacement are pairwise independent with mean
1/K, so the fraction of equal pairs over the N pairs of a periodic L x L
lattice has standard error sqrt(p (1 - p) / N).  Per-row and per-column
species counts are multinomial(L, 1/K), so their chi-square statistic over
the lattice has L (K - 1) degrees of freedom.  A generator whose draws are
correlated between sites (the paper's Metal Mersenne Twister showed vertical
stripes) breaks one of these.
"""
from __future__ import annotations

import numpy as np


def equal_pair_fraction(g: np.ndarray, dy: int, dx: int) -> float:
    """Fraction of sites equal to their periodic neighbour at (dy, dx)."""
    return float((g == np.roll(np.roll(g, -dy, 0), -dx, 1)).mean())


def line_chi2(g: np.ndarray, K: int, axis: int):
    """(statistic, degrees of freedom) of the per-row (axis=1) or per-column
    (axis=0) species counts against the uniform law."""
    L = g.shape[axis]
    e = L / K
    stat = 0.0
    for s in range(K):
        n = (g == s).sum(axis=axis).astype(np.float64)
        stat += float(((n - e) ** 2 / e).sum())
    return stat, g.shape[1 - axis] * (K - 1)


def screen(g: np.ndarray, K: int, z: float = 5.0):
    """Failed checks (empty list = pass) of a 2-D lattice whose sites should
    be i.i.d. uniform over 0..K-1: equal-pair fractions horizontally at
    distances 1..8 (the block schedule's quads span 8 columns), vertically
    at 1..4 and diagonally at (1, 1), (1, -1), each within z standard
    errors of 1/K; row and column chi-square within z standard deviations
    (sqrt(2 df)) of df."""
    p = 1.0 / K
    se = np.sqrt(p * (1 - p) / g.size)
    bad = []
    shifts = [(0, d) for d in range(1, 9)] + [(d, 0) for d in range(1, 5)]
    shifts += [(1, 1), (1, -1)]
    for dy, dx in shifts:
        f = equal_pair_fraction(g, dy, dx)
        if abs(f - p) > z * se:
            bad.append(f"equal pairs at ({dy},{dx}): {f:.5f} vs {p:.5f} "
                       f"(se {se:.2e})")
    for axis, name in ((1, "rows"), (0, "columns")):
        stat, df = line_chi2(g, K, axis)
        if abs(stat - df) > z * np.sqrt(2 * df):
            bad.append(f"{name} chi2 {stat:.1f} vs df {df}")
    return bad
