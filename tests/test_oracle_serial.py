"""Pins for the oracle's exact serial SSA, part (a) (test infrastructure).

The whole-lattice SSA (eqs. totalrate, skeleton) must reproduce the master
equation of eq. generator: on tiny lattices the replica means of the count
observables must lie within 3 standard errors of p0 exp(tQ) (Q enumerated
independently in oracle/exact.py), and on a non-interacting lattice within 3
standard errors of the single-site closed form.
"""
import numpy as np
import pytest

from oracle import exact
from _exact_stats import assert_within_3se, delta_state, moments


def _serial_obs(orc, model, lat0, times, R, seed=0):
    T = float(times[-1]) + 1e-9
    out = np.zeros((R, len(times), 7))
    for r in range(R):
        _, o, _ = orc.ssa_serial(model, lat0, T, seed, r, times)
        out[r] = o
    return out


CASES = [
    # kind, Lx, Ly, params, initial state, observed columns
    ("flip", 3, 3, dict(k_a=1.0, k_d=1.0, J=1.0, h=0.0, beta=1.0), 0, (1, 4)),
    ("flip", 2, 2, dict(k_a=0.7, k_d=1.3, J=2.0, h=-1.0, beta=1.0), 1, (1, 4)),
    ("flip", 8, 1, dict(k_a=1.0, k_d=2.0, J=1.5, h=-0.5, beta=1.2), 0, (1, 4)),
    ("zgb", 3, 2, dict(y=0.45, k_r=3.0, D=1.5), 0, (0, 1, 2, 6)),
    ("zgb", 2, 2, dict(y=0.6, k_r=5.0, D=0.0), 0, (0, 1, 2, 6)),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}{c[1]}x{c[2]}" for c in CASES])
def test_serial_matches_master_equation(orc, case):
    kind, Lx, Ly, params, s0, cols = case
    model = orc.Model(kind, Lx, Ly, **params)
    lat0 = np.full(model.N, s0, np.uint8)
    times = np.array([0.15, 0.5, 1.2, 2.5])
    R = 3000
    sample = _serial_obs(orc, model, lat0, times, R)
    Q = exact.generator(kind, model.params[:5 if kind == "flip" else 3], Lx, Ly)
    ov = exact.observable_vectors(kind, Lx, Ly)
    p0 = delta_state(kind, lat0)
    for k, t in enumerate(times):
        mean, var = moments(exact.propagate(p0, Q, t), ov)
        assert_within_3se(sample[:, k, :], mean, var, cols, label=(kind, Lx, Ly, t))


def test_serial_noninteracting_closed_form(orc):
    """J = 0: every site is an independent two-state chain."""
    k_a, k_d = 1.0, 2.0
    model = orc.Model("flip", 32, 32, k_a=k_a, k_d=k_d, J=0.0)
    times = np.array([0.1, 0.3, 0.6, 1.0, 2.0, 4.0])
    R = 32
    sample = _serial_obs(orc, model, np.zeros(model.N, np.uint8), times, R)
    cov = sample[:, :, 1] / model.N
    th = exact.single_site_coverage(k_a, k_d, 0.0, times)
    se = np.sqrt(th * (1 - th) / (model.N * R))
    assert np.all(np.abs(cov.mean(axis=0) - th) <= 3 * se), (cov.mean(axis=0), th, se)


def test_serial_monomer_only_closed_form(orc):
    """Reaction model with y = 1: only A adsorption at rate 1 per empty site,
    so the A coverage is 1 - exp(-t) exactly."""
    model = orc.Model("zgb", 16, 16, y=1.0, k_r=1000.0, D=10.0)
    times = np.array([0.2, 0.7, 1.5, 3.0])
    R = 32
    sample = _serial_obs(orc, model, np.zeros(model.N, np.uint8), times, R)
    th = 1.0 - np.exp(-times)
    se = np.sqrt(th * (1 - th) / (model.N * R))
    assert np.all(sample[:, :, 2] == 0)
    assert np.all(np.abs(sample[:, :, 1].mean(axis=0) / model.N - th) <= 3 * se)


def test_serial_absorbing_state_stops(orc):
    """No empty site and no A-B pair: total rate zero, nothing happens."""
    model = orc.Model("zgb", 4, 4, y=0.5, k_r=10.0, D=1.0)
    lat = np.full(16, 2, np.uint8)
    out, obs, ev = orc.ssa_serial(model, lat, 5.0, 0, 0, [1.0, 5.0])
    assert ev == 0 and np.all(out == 2) and obs[1, 2] == 16
