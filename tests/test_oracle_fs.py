"""Pins for the oracle's fractional-step scheme, part (b) (test infrastructure).

What the paper and the mathematics fix, independently of the oracle's code:

* On tiny lattices the fractional-step chain has the law of the exact split
  propagator p0 prod_w exp(d_w Q_{c_w}) (eqs. lie, strang with eq. exact):
  replica means within 3 standard errors.  The chosen step is large enough that
  the split law and the serial law are more than 6 standard errors apart, so
  the check tells the two apart.
* With J = 0 the commutator [L^E, L^O] vanishes (Sec. 4.1, eq. lieboundary:
  only boundary terms survive and those vanish without interaction), so the
  scheme is exact for any step: the single-site closed form must hold.
* The Arrhenius dynamics is reversible with respect to its Gibbs measure
  (Sec. 7); each colour generator is then self-adjoint for the same measure,
  so every window preserves it and the scheme's equilibrium is the exact Gibbs
  measure even at dt = 1 (the step the paper's 1D phase diagram uses).  Checked
  against the transfer matrix (1D) and brute-force Gibbs sums (2D).
* The schedule: Lie is first order and Strang second order (eqs. error and
  error2), checked deterministically on the split propagator built from the
  oracle's own window list.
* The decomposition checker enforces closure independence (Sec. 2.1 remark).
"""
import numpy as np
import pytest

import oracle as _o
from oracle import exact
from _exact_stats import assert_within_3se, delta_state, moments


def _fs_obs(orc, model, lat0, bx, by, cmap, ncol, split, dt, T, R, seed=0):
    cols, durs, ends = orc.schedule(split, ncol, dt, T, seed)
    out = []
    for r in range(R):
        res = orc.fs_run(model, lat0, bx, by, cmap, ncol, cols, durs, seed, r, observe_flags=ends)
        out.append(res["obs"])
    return np.array(out, dtype=np.float64), cols, durs, ends


def _colour_generators(kind, params, Lx, Ly, bx, by, cmap, ncol, sparse=False):
    return [exact.generator(kind, params, Lx, Ly, owner=exact.site_owner_by_colour(Lx, Ly, bx, by, cmap, c),
                            sparse=sparse) for c in range(ncol)]


SPLIT_CASES = [
    # kind, Lx, Ly, params, bx, by, colour map, colours, split, dt, T, cols, discriminating
    ("flip", 2, 4, dict(k_a=1.0, k_d=1.0, J=1.5, h=-0.5, beta=1.0), 1, 2, [0, 1, 1, 0], 2, _o.LIE, 1.0, 2.0,
     (1, 4), True),
    ("flip", 2, 4, dict(k_a=1.0, k_d=1.0, J=1.5, h=-0.5, beta=1.0), 1, 2, [0, 1, 1, 0], 2, _o.STRANG, 1.0, 2.0,
     (1, 4), False),
    ("flip", 3, 3, dict(k_a=1.0, k_d=0.5, J=1.0, h=-0.3, beta=1.0), 1, 1,
     [(i + j) % 3 for j in range(3) for i in range(3)], 3, _o.STRANG, 0.5, 1.5, (1, 4), False),
    ("zgb", 4, 2, dict(y=0.45, k_r=4.0, D=2.0), 2, 1, None, 4, _o.STRANG, 0.25, 0.5, (0, 1, 2, 6), False),
    ("zgb", 4, 2, dict(y=0.3, k_r=2.0, D=0.0), 2, 1, None, 4, _o.LIE, 0.5, 1.0, (0, 1, 2, 6), False),
]


@pytest.mark.parametrize("case", SPLIT_CASES,
                         ids=[f"{c[0]}{c[1]}x{c[2]}-{['lie', 'strang', 'random'][c[8]]}" for c in SPLIT_CASES])
def test_fs_matches_split_propagator(orc, case):
    kind, Lx, Ly, params, bx, by, cmap, ncol, split, dt, T, cols_obs, disc = case
    model = orc.Model(kind, Lx, Ly, **params)
    if cmap is None:
        cmap = orc.colour_map(model, bx, by, ncol)
    cmap = np.asarray(cmap, np.int32)
    assert orc.decomp_check(model, bx, by, cmap, ncol) == 0
    lat0 = np.zeros(model.N, np.uint8)
    R = 3000
    sample, cols, durs, ends = _fs_obs(orc, model, lat0, bx, by, cmap, ncol, split, dt, T, R)
    pr = model.params[:5 if kind == "flip" else 3]
    sparse = kind == "zgb"
    Qc = _colour_generators(kind, pr, Lx, Ly, bx, by, cmap, ncol, sparse)
    Q = exact.generator(kind, pr, Lx, Ly, sparse=sparse)
    ov = exact.observable_vectors(kind, Lx, Ly)
    p = delta_state(kind, lat0)
    step_ends = np.nonzero(ends)[0]
    start = 0
    for k, w_end in enumerate(step_ends):
        p = exact.split_propagate(p, Qc, cols[start:w_end + 1], durs[start:w_end + 1])
        start = w_end + 1
        mean, var = moments(p, ov)
        assert_within_3se(sample[:, k, :], mean, var, cols_obs, label=(kind, k))
    if disc:
        me, _ = moments(exact.propagate(delta_state(kind, lat0), Q, T), ov)
        ms, vs = moments(p, ov)
        assert max(abs(ms[c] - me[c]) / np.sqrt(vs[c] / R) for c in cols_obs) > 6.0


def test_fs_noninteracting_is_exact_for_any_step(orc):
    k_a, k_d = 1.0, 2.0
    model = orc.Model("flip", 32, 32, k_a=k_a, k_d=k_d, J=0.0)
    cmap = orc.colour_map(model, 8, 8, 2)
    for split in (_o.LIE, _o.STRANG):
        R = 32
        sample, _, _, _ = _fs_obs(orc, model, np.zeros(model.N, np.uint8), 8, 8, cmap, 2, split, 1.0, 4.0, R)
        times = np.arange(1, 5, dtype=np.float64)
        th = exact.single_site_coverage(k_a, k_d, 0.0, times)
        se = np.sqrt(th * (1 - th) / (model.N * R))
        cov = sample[:, :, 1].mean(axis=0) / model.N
        assert np.all(np.abs(cov - th) <= 3 * se), (split, cov, th, se)


def _time_avg(sample, burn, N):
    cov = sample[:, burn:, 1].mean(axis=1) / N
    bond = sample[:, burn:, 4].mean(axis=1) / N
    return cov, bond


@pytest.mark.parametrize("split", [_o.LIE, _o.STRANG])
def test_fs_equilibrium_is_gibbs_1d(orc, split):
    J, h, beta = 1.0, -0.5, 1.0
    N = 32
    model = orc.Model("flip", N, 1, k_a=1.0, k_d=1.0, J=J, h=h, beta=beta)
    cmap = orc.colour_map(model, 4, 1, 2)
    R = 32
    sample, _, _, _ = _fs_obs(orc, model, np.zeros(N, np.uint8), 4, 1, cmap, 2, split, 1.0, 400.0, R)
    cov, bond = _time_avg(sample, 40, N)
    ec, eb = exact.transfer_matrix_1d(N, J, h, beta)
    for got, ref in ((cov, ec), (bond, eb)):
        se = got.std(ddof=1) / np.sqrt(R)
        assert abs(got.mean() - ref) <= 3 * se, (got.mean(), ref, se)


def test_fs_equilibrium_is_gibbs_2d(orc):
    J, h, beta = 0.8, -1.0, 1.0
    model = orc.Model("flip", 4, 4, k_a=1.0, k_d=1.0, J=J, h=h, beta=beta)
    cmap = orc.colour_map(model, 2, 2, 2)
    R = 32
    sample, _, _, _ = _fs_obs(orc, model, np.zeros(16, np.uint8), 2, 2, cmap, 2, _o.LIE, 1.0, 600.0, R)
    cov, bond = _time_avg(sample, 50, 16)
    ec, eb = exact.exact_equilibrium_small(4, 4, J, h, beta)
    for got, ref in ((cov, ec), (bond, eb)):
        se = got.std(ddof=1) / np.sqrt(R)
        assert abs(got.mean() - ref) <= 3 * se, (got.mean(), ref, se)


def test_schedule_orders_of_accuracy(orc):
    """||p_FS(T) - p(T)||_1 halves (Lie) or quarters (Strang) when dt halves."""
    kind, Lx, Ly, bx, by, cmap = "flip", 2, 4, 1, 2, np.array([0, 1, 1, 0], np.int32)
    model = orc.Model(kind, Lx, Ly, k_a=1.0, k_d=1.0, J=1.5, h=-0.5, beta=1.0)
    Q = exact.generator(kind, model.params, Lx, Ly)
    Qc = _colour_generators(kind, model.params, Lx, Ly, bx, by, cmap, 2)
    p0 = delta_state(kind, np.zeros(model.N, np.uint8))
    T = 1.0
    pe = exact.propagate(p0, Q, T)
    for split, order in ((_o.LIE, 1), (_o.STRANG, 2)):
        errs = []
        for dt in (0.1, 0.05, 0.025):
            cols, durs, _ = orc.schedule(split, 2, dt, T)
            errs.append(np.abs(exact.split_propagate(p0, Qc, cols, durs) - pe).sum())
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(np.abs(rates - order) < 0.15), (split, errs, rates)


def test_schedule_window_lists(orc):
    c, d, e = orc.schedule(_o.LIE, 2, 0.1, 0.3)
    assert list(c) == [0, 1] * 3 and np.all(d == 0.1) and list(e) == [0, 1] * 3
    c, d, e = orc.schedule(_o.STRANG, 2, 0.1, 0.2)
    assert list(c) == [0, 1, 0, 0, 1, 0] and list(d) == [0.05, 0.1, 0.05] * 2
    c, d, e = orc.schedule(_o.STRANG, 4, 0.2, 0.2)
    assert list(c) == [0, 1, 2, 3, 2, 1, 0] and list(d) == [0.1, 0.1, 0.1, 0.2, 0.1, 0.1, 0.1]
    assert list(e) == [0, 0, 0, 0, 0, 0, 1]
    c, d, e = orc.schedule(_o.RANDOM, 2, 0.5, 50.0)
    assert len(c) == 200 and np.all(d == 0.5) and set(c) == {0, 1}
    assert abs(c.mean() - 0.5) < 0.15
    with pytest.raises(ValueError):
        orc.schedule(_o.LIE, 2, 0.3, 1.0)


def test_decomposition_checker(orc):
    flip = orc.Model("flip", 16, 16)
    zgb = orc.Model("zgb", 16, 16)
    for b in (1, 2, 4):
        assert orc.decomp_check(flip, b, b, orc.colour_map(flip, b, b, 2), 2) == 0
    # pair events reach across the block edge: 2 colours are not independent
    for b in (2, 4):
        assert orc.decomp_check(zgb, b, b, orc.colour_map(zgb, b, b, 2), 2) == -4
        assert orc.decomp_check(zgb, b, b, orc.colour_map(zgb, b, b, 4), 4) == 0
    assert orc.decomp_check(zgb, 1, 1, orc.colour_map(zgb, 1, 1, 4), 4) == -4
    # a single colour is never independent, blocks must tile the lattice
    assert orc.decomp_check(flip, 4, 4, np.zeros(16, np.int32), 1) == -4
    assert orc.decomp_check(flip, 5, 4, np.zeros(16, np.int32), 2) == -1


def test_fs_matches_serial_at_small_step_reaction(orc):
    """No exact solution for the reaction model: at dt = 0.01 the scheme and
    the serial SSA must agree statistically (species coverages at T = 1)."""
    model = orc.Model("zgb", 16, 16, y=0.5, k_r=20.0, D=2.0)
    cmap = orc.colour_map(model, 4, 4, 4)
    R = 48
    lat0 = np.zeros(model.N, np.uint8)
    fs, _, _, _ = _fs_obs(orc, model, lat0, 4, 4, cmap, 4, _o.STRANG, 0.01, 1.0, R)
    fs_end = fs[:, -1, :3] / model.N
    ser = np.array([orc.ssa_serial(model, lat0, 1.0 + 1e-9, 0, 1000 + r, [1.0])[1][0, :3] for r in range(R)])
    ser = ser / model.N
    for c in range(3):
        se = np.sqrt(fs_end[:, c].var(ddof=1) / R + ser[:, c].var(ddof=1) / R)
        assert abs(fs_end[:, c].mean() - ser[:, c].mean()) <= 3 * se
