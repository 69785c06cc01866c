"""Helpers for the statistical oracle pins: exact means and variances of the
count observables under a distribution over configurations, and the 3-sigma
comparison of replica means against them."""
import numpy as np

from oracle import exact


def delta_state(kind, lattice):
    K = 3 if kind == "zgb" else 2
    p0 = np.zeros(K ** len(lattice))
    p0[exact.state_index(tuple(int(v) for v in lattice), K)] = 1.0
    return p0


def moments(p, obsvec):
    mean = p @ obsvec
    var = p @ (obsvec ** 2) - mean ** 2
    return mean, np.maximum(var, 0.0)


def assert_within_3se(sample, mean, var, cols, label=""):
    """sample: [R, 7] replica observations; mean/var: exact moments [7]."""
    R = sample.shape[0]
    for c in cols:
        se = np.sqrt(var[c] / R)
        got = sample[:, c].mean()
        if var[c] == 0:
            assert got == mean[c], (label, c, got, mean[c])
        else:
            assert abs(got - mean[c]) <= 3.0 * se, (label, c, got, mean[c], se)
