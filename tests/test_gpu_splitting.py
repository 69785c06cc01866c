"""Splitting error of the fractional-step scheme at full size (needs a GPU).

The 1024^2 Ising-type lattice (spin flip, Arrhenius rates, h = 0, beta = 1,
16x16 blocks, Bernoulli(1/2) start) at J = 0.5 and J = 1: coverage theta =
#occupied / N and the energy density e = -J #(occupied nearest-neighbour
bonds) / N at t = 1, 2, 5, 10, over 32 replicas of the exact serial SSA (the
oracle, on the host cores) and 32 replicas of the fractional-step scheme on
the GPU for Lie and Strang at dt = 0.01, 0.1, 1.  The error of each scheme is
the difference of the replica means in units of the combined standard
error.  At dt = 0.01 the schemes agree with the exact dynamics within 4
standard errors (all times, both observables, both couplings); the full table
is printed.
"""
import concurrent.futures
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L, B, T = 1024, 16, 10.0
TIMES = (1.0, 2.0, 5.0, 10.0)
R = 32


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


def _serial(orc, J):
    """theta and e at TIMES for R replicas of the exact serial SSA."""
    m = orc.Model("flip", L, L, k_a=1.0, k_d=1.0, J=J, h=0.0, beta=1.0)

    def one(r):
        lat0 = orc.init_bernoulli(L * L, 0.5, 7, r)
        _, obs, _ = orc.ssa_serial(m, lat0, T + 1e-9, 7, r, list(TIMES))
        return obs[:, 1] / (L * L), -J * obs[:, 4] / (L * L)

    workers = min(16, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:  # the oracle's C releases the GIL
        out = list(ex.map(one, range(R)))
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


def _fs(F, ctx, J, split, dt):
    per = 2 if split == 0 else 3
    theta = np.zeros((R, len(TIMES)))
    energy = np.zeros((R, len(TIMES)))
    for r in range(R):
        s = F.Sim(ctx, "flip", L, L, (1.0, 1.0, J, 0.0, 1.0), b=B, n_colours=2, dt=dt, T=T, split=split, seed=7,
                  replica=r)
        s.init(1, 0.5)
        done = 0
        for k, t in enumerate(TIMES):
            target = int(round(t / dt)) * per
            s.advance(target - done)
            done = target
            o = s.observe()
            theta[r, k] = o["count"][1] / (L * L)
            energy[r, k] = -J * o["bonds_equal"][1] / (L * L)
        s.close()
    return theta, energy


def _z(a, b):
    se = np.sqrt(a.var(axis=0, ddof=1) / len(a) + b.var(axis=0, ddof=1) / len(b))
    return (a.mean(axis=0) - b.mean(axis=0)) / np.maximum(se, 1e-300), a.mean(axis=0) - b.mean(axis=0)


@pytest.mark.parametrize("J", [0.5, 1.0])
def test_splitting_error_against_serial_ssa(F, orc, J):
    ctx = F.fskmc_ctx_create(0)
    F.fskmc_ctx_set_persistent(ctx, 100000)  # the resident sweep, as the bench times it
    try:
        th_ex, en_ex = _serial(orc, J)
        print(f"\nJ = {J}: exact serial SSA, {R} replicas: theta {np.round(th_ex.mean(0), 5)}, "
              f"e {np.round(en_ex.mean(0), 5)} at t = {TIMES}")
        for split, name in ((0, "Lie"), (1, "Strang")):
            for dt in (0.01, 0.1, 1.0):
                th, en = _fs(F, ctx, J, split, dt)
                zt, dth = _z(th, th_ex)
                ze, den = _z(en, en_ex)
                print(f"J = {J} {name:6s} dt = {dt:<5}: theta error {np.array2string(dth, precision=5)} "
                      f"({np.array2string(zt, precision=1)} SE); e error {np.array2string(den, precision=5)} "
                      f"({np.array2string(ze, precision=1)} SE)")
                if dt == 0.01:
                    assert np.all(np.abs(zt) < 4) and np.all(np.abs(ze) < 4), (J, name, zt, ze)
    finally:
        F.fskmc_ctx_destroy(ctx)
