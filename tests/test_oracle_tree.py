"""Pins for the oracle's sum tree and event selection (test infrastructure).

The tree computes the total rate (eq. totalrate) and the descent selects a
site with probability c(x)/lambda (eq. skeleton).  Checked against exact
rational arithmetic and brute-force frequencies, not against itself.
"""
import math
from fractions import Fraction

import numpy as np

EPS = 2.0 ** -53


def _leaves(rng, n, pzero):
    v = rng.exponential(1.0, n) * np.exp(rng.uniform(-6, 6, n))
    v[rng.random(n) < pzero] = 0.0
    return v


def test_root_is_the_sum(orc):
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 7, 64, 100, 256, 1000, 1024):
        v = _leaves(rng, n, 0.3)
        _, root, _ = orc.tree_select(v, 0.5)
        exact = math.fsum(v)
        assert abs(root - exact) <= max(n - 1, 1) * EPS * exact + 1e-300


def test_selection_brackets_the_target(orc):
    """The selected leaf i satisfies S_i <= V*R < S_{i+1} up to rounding,
    with S_i the exact prefix sum of the leaves before i, and has a positive rate."""
    rng = np.random.default_rng(4)
    for trial in range(300):
        n = int(rng.integers(1, 300))
        v = _leaves(rng, n, float(rng.uniform(0, 0.9)))
        if v.sum() == 0:
            v[int(rng.integers(0, n))] = 1.0
        V = float(rng.random()) if trial % 10 else 1.0 - EPS
        i, root, resid = orc.tree_select(v, V)
        assert 0 <= i < n and v[i] > 0
        pref = [Fraction(0)]
        for x in v:
            pref.append(pref[-1] + Fraction(float(x)))
        tg = Fraction(V) * Fraction(root)
        slack = Fraction(4 * n) * Fraction(EPS) * pref[-1]
        assert pref[i] - slack <= tg <= pref[i + 1] + slack
        # the residual is the target minus everything to the left of leaf i
        assert abs(Fraction(resid) - (tg - pref[i])) <= slack


def test_selection_frequencies_on_a_grid(orc):
    """Over a uniform grid of V the fraction of points mapping to leaf i is
    c_i / lambda to within the grid resolution."""
    rng = np.random.default_rng(5)
    for n in (5, 16, 37):
        v = _leaves(rng, n, 0.25)
        v[0] = max(v[0], 0.1)
        M = 20000
        counts = np.zeros(n, int)
        for j in range(M):
            i, _, _ = orc.tree_select(v, (j + 0.5) / M)
            counts[i] += 1
        p = v / v.sum()
        assert np.all(np.abs(counts / M - p) <= 2.0 / M + 1e-12)
        assert np.all(counts[v == 0] == 0)


def test_zero_total_selects_nothing(orc):
    i, root, _ = orc.tree_select(np.zeros(10), 0.3)
    assert i == -1 and root == 0.0


def test_trailing_zeros_never_selected_at_the_top(orc):
    """V just below 1 must not fall through into empty trailing leaves."""
    for n in (3, 9, 100):
        v = np.zeros(n)
        v[0] = 0.1
        v[1] = 0.2
        i, _, _ = orc.tree_select(v, 1.0 - EPS)
        assert i == 1
