"""Pins for the oracle's conserved spin-exchange (Kawasaki) model (Sec. 2, the
diffusion example), independent of its code:

* the rate table equals an independent enumeration of the exchange events
  (oracle/exact.py) for all 32 neighbourhoods of states {0, 1};
* the particle number is invariant, exactly, under the serial SSA and the
  fractional-step scheme (the update exchanges two sites);
* the serial SSA follows the master equation p0 exp(tQ) on a 3x3 torus;
* at J = 0 the dynamics is the symmetric exclusion process, whose one-point
  function solves the lattice heat equation exactly:
  E sigma_t = exp(t D/4 (A - 4 I)) sigma_0 (A the torus adjacency matrix);
* the fractional-step scheme (4 colours, pair events) follows the exact split
  propagator on a 4x2 lattice.
"""
import math

import numpy as np
import scipy.linalg

import oracle as _o
from oracle import exact
from _exact_stats import assert_within_3se, delta_state, moments

PRM = dict(D=2.0, J=1.5, beta=1.0)


def test_rate_table_vs_event_enumeration(orc):
    D, J, beta = 1.7, 0.8, 1.3
    m = orc.Model("kawasaki", 3, 3, D=D, J=J, beta=beta)
    tab = orc.rate_table(m).reshape(243, 14)
    centre, nbr = 4, {0: 5, 1: 3, 2: 7, 3: 1}  # E, W, N, S of (1,1) on a 3x3 torus
    for bits in range(32):
        conf = [0] * 9
        conf[centre] = bits & 1
        for d in range(4):
            conf[nbr[d]] = (bits >> (d + 1)) & 1
        pat = conf[centre] + sum(conf[nbr[d]] * 3 ** (d + 1) for d in range(4))
        evs = [e for e in exact.events("kawasaki", (D, J, beta), 3, 3, tuple(conf)) if e[0] == centre]
        total = math.fsum(e[1] for e in evs)
        assert abs(tab[pat, 13] - total) <= 8 * math.ulp(max(total, 1e-300)), bits
        assert all(tab[pat, c] == 0.0 for c in range(9)), bits
        got = sorted((tab[pat, 9 + d], nbr[d]) for d in range(4) if tab[pat, 9 + d] > 0)
        want = sorted((e[1], [q for q in range(9) if e[2][q] == 1 and conf[q] == 0][0]) for e in evs)
        assert [q for _, q in got] == [q for _, q in want], bits
        for (a, _), (b, _) in zip(got, want):
            assert abs(a - b) <= 4 * math.ulp(b), bits


def test_particle_number_conserved(orc):
    m = orc.Model("kawasaki", 16, 16, D=4.0, J=0.5, beta=1.0)
    rng = np.random.default_rng(4)
    lat0 = (rng.random(m.N) < 0.4).astype(np.uint8)
    n0 = int(lat0.sum())
    lat, obs, ev = orc.ssa_serial(m, lat0, 5.0, 0, 1, [1.0, 2.5, 5.0])
    assert ev > 300 and int(lat.sum()) == n0 and np.all(obs[:, 1] == n0)
    cmap = orc.colour_map(m, 4, 4, 4)
    cols, durs, ends = orc.schedule(_o.STRANG, 4, 0.5, 5.0)
    res = orc.fs_run(m, lat0, 4, 4, cmap, 4, cols, durs, 0, 2, observe_flags=ends)
    assert res["events"] > 300 and int(res["lattice"].sum()) == n0
    assert np.all(res["obs"][:, 1] == n0)


def test_serial_matches_master_equation(orc):
    Lx, Ly = 3, 3
    m = orc.Model("kawasaki", Lx, Ly, **PRM)
    lat0 = np.array([1, 1, 1, 1, 0, 0, 0, 0, 0], np.uint8)
    times = np.array([0.2, 0.6, 1.5, 3.0])
    R = 3000
    sample = np.zeros((R, len(times), 7))
    for r in range(R):
        sample[r] = orc.ssa_serial(m, lat0, times[-1] + 1e-9, 0, r, times)[1]
    Q = exact.generator("kawasaki", m.params[:3], Lx, Ly)
    ov = exact.observable_vectors("kawasaki", Lx, Ly)
    p0 = delta_state("kawasaki", lat0)
    for k, t in enumerate(times):
        mean, var = moments(exact.propagate(p0, Q, t), ov)
        assert_within_3se(sample[:, k, :], mean, var, (3, 4), label=("kawasaki", t))


def test_exclusion_process_one_point_function(orc):
    """J = 0: mean occupation of every site = heat kernel applied to sigma_0."""
    L, D = 6, 2.0
    m = orc.Model("kawasaki", L, L, D=D, J=0.0, beta=1.0)
    lat0 = np.zeros(L * L, np.uint8)
    for y in range(2):
        for x in range(3):
            lat0[y * L + x] = 1
    A = np.zeros((L * L, L * L))
    for s in range(L * L):
        for q in exact._neighbours(L, L, 2, s):
            A[s, q] += 1
    t = 0.8
    want = scipy.linalg.expm(t * D / 4.0 * (A - 4.0 * np.eye(L * L))) @ lat0.astype(float)
    R = 4000
    occ = np.zeros(L * L)
    for r in range(R):
        lat, _, _ = orc.ssa_serial(m, lat0, t, 0, 100 + r, [t])
        occ += lat
    got = occ / R
    se = np.sqrt(np.maximum(want * (1 - want), 1e-12) / R)
    assert np.all(np.abs(got - want) <= 4 * se + 1e-12), np.max(np.abs(got - want) / se)


def test_fs_matches_split_propagator(orc):
    Lx, Ly, bx, by = 4, 2, 2, 1
    m = orc.Model("kawasaki", Lx, Ly, **PRM)
    cmap = orc.colour_map(m, bx, by, 4)
    assert orc.decomp_check(m, bx, by, cmap, 4) == 0
    lat0 = np.array([1, 1, 0, 0, 1, 0, 1, 0], np.uint8)
    cols, durs, ends = orc.schedule(_o.STRANG, 4, 0.5, 1.0)
    R = 3000
    sample = np.array([orc.fs_run(m, lat0, bx, by, cmap, 4, cols, durs, 0, r, observe_flags=ends)["obs"]
                       for r in range(R)], dtype=np.float64)
    Qc = [exact.generator("kawasaki", m.params[:3], Lx, Ly,
                          owner=exact.site_owner_by_colour(Lx, Ly, bx, by, cmap, c)) for c in range(4)]
    ov = exact.observable_vectors("kawasaki", Lx, Ly)
    p = delta_state("kawasaki", lat0)
    start = 0
    for k, w_end in enumerate(np.nonzero(ends)[0]):
        p = exact.split_propagate(p, Qc, cols[start:w_end + 1], durs[start:w_end + 1])
        start = w_end + 1
        mean, var = moments(p, ov)
        assert_within_3se(sample[:, k, :], mean, var, (3, 4), label=("kawasaki-fs", k))
