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
* The random schedule (Sec. 3.1): its replica law is the averaged one-window
  propagator; its mean local error is the (A1 - A2)^2 term of Sec. 4.1 while
  Lie's is the commutator, so Lie wins at equal step and more so for larger
  cells (eq. pcscompare).
"""
import numpy as np
import pytest
import scipy.linalg

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


def test_fs_random_schedule_matches_averaged_propagator(orc):
    """Random schedule (Sec. 3.1, eq. SLPCS): every replica draws its own
    colour sequence, uniform and independent per window, so the law over
    replicas is p0 M^w with M = (1/K) sum_c exp(dt Q_c), the one-window form
    of the averaged operator (eq. averaged).  The step is large enough that
    this law differs from the serial one and from the Lie scheme's by more
    than 6 standard errors."""
    kind, Lx, Ly, bx, by, ncol = "flip", 2, 4, 1, 2, 2
    cmap = np.array([0, 1, 1, 0], np.int32)
    model = orc.Model(kind, Lx, Ly, k_a=1.0, k_d=1.0, J=1.5, h=-0.5, beta=1.0)
    dt, T, R = 1.0, 2.0, 3000
    lat0 = np.zeros(model.N, np.uint8)
    sample, seqs = [], set()
    for r in range(R):
        cols, durs, ends = orc.schedule(_o.RANDOM, ncol, dt, T, 0, r)
        seqs.add(tuple(cols))
        sample.append(orc.fs_run(model, lat0, bx, by, cmap, ncol, cols, durs, 0, r, observe_flags=ends)["obs"])
    sample = np.array(sample, dtype=np.float64)
    assert len(seqs) == 2 ** 4        # 4 windows, every colour sequence occurs
    Qc = _colour_generators(kind, model.params, Lx, Ly, bx, by, cmap, ncol)
    M = sum(scipy.linalg.expm(dt * q) for q in Qc) / ncol
    ov = exact.observable_vectors(kind, Lx, Ly)
    p = delta_state(kind, lat0)
    for k in range(int(T / dt)):
        for _ in range(ncol):
            p = p @ M
        mean, var = moments(p, ov)
        assert_within_3se(sample[:, k, :], mean, var, (1, 4), label=("random", k))
    ms, vs = moments(p, ov)
    me, _ = moments(exact.propagate(delta_state(kind, lat0), exact.generator(kind, model.params, Lx, Ly), T), ov)
    cols, durs, _ = orc.schedule(_o.LIE, ncol, dt, T)
    ml, _ = moments(exact.split_propagate(delta_state(kind, lat0), Qc, cols, durs), ov)
    for other in (me, ml):
        assert max(abs(ms[c] - other[c]) / np.sqrt(vs[c] / R) for c in (1, 4)) > 6.0


def test_random_schedule_colours_uniform_and_independent(orc):
    """Colour draws of the random schedule: uniform over K colours, the pair
    of consecutive windows uniform over K^2 (independence), chi-square at the
    0.1% level; the replica key changes the sequence."""
    from scipy.stats import chisquare
    for K in (2, 4):
        cols = np.concatenate([orc.schedule(_o.RANDOM, K, 0.5, 100.0, 0, r)[0] for r in range(20)])
        assert chisquare(np.bincount(cols, minlength=K)).pvalue > 1e-3
        pairs = cols[:-1] * K + cols[1:]
        assert chisquare(np.bincount(pairs, minlength=K * K)).pvalue > 1e-3
    a = orc.schedule(_o.RANDOM, 2, 0.5, 100.0, 0, 0)[0]
    b = orc.schedule(_o.RANDOM, 2, 0.5, 100.0, 0, 1)[0]
    c = orc.schedule(_o.RANDOM, 2, 0.5, 100.0, 1, 0)[0]
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_random_schedule_mean_local_error():
    """Sec. 4.1: averaged over the colours of two windows, the local error
    against exp(dt (A1 + A2)) is (1/4)(A1 - A2)^2 dt^2 + O(dt^3); the Lie
    product's is (1/2)[A1, A2] dt^2 + O(dt^3).  Checked on the coverage of a
    2x4 lattice: the remainder divided by dt^2 shrinks linearly with dt."""
    Lx, Ly, bx, by = 2, 4, 1, 2
    prm = (1.0, 1.0, 1.5, -0.5, 1.0)
    cmap = np.array([0, 1, 1, 0], np.int32)
    A = [exact.generator("flip", prm, Lx, Ly, owner=exact.site_owner_by_colour(Lx, Ly, bx, by, cmap, c))
         for c in range(2)]
    f = exact.observable_vectors("flip", Lx, Ly)[:, 1] / (Lx * Ly)
    lead_rnd = 0.25 * (A[0] - A[1]) @ ((A[0] - A[1]) @ f)
    lead_lie = 0.5 * (A[0] @ (A[1] @ f) - A[1] @ (A[0] @ f))
    assert np.abs(lead_rnd).max() > 0.1 and np.abs(lead_lie).max() > 0.1
    rem = {"rnd": [], "lie": []}
    for dt in (0.02, 0.01, 0.005):
        E = [scipy.linalg.expm(dt * a) for a in A]
        ref = scipy.linalg.expm(dt * (A[0] + A[1])) @ f
        rnd = 0.25 * sum(E[i] @ (E[j] @ f) for i in range(2) for j in range(2)) - ref
        lie = E[0] @ (E[1] @ f) - ref
        rem["rnd"].append(np.abs(rnd / dt ** 2 - lead_rnd).max())
        rem["lie"].append(np.abs(lie / dt ** 2 - lead_lie).max())
    for k, r in rem.items():
        ratios = np.array(r[:-1]) / np.array(r[1:])
        assert np.all(np.abs(ratios - 2.0) < 0.2), (k, r)


def test_pcs_compare_lie_allows_larger_step(orc):
    """Sec. 4.1, eqs. lietimestep, randomtimestep, pcscompare: the Lie error
    carries the commutator, which only the cell boundaries feed (eq.
    lieboundary, O(1/q) for cells of q sites), while the random schedule's
    mean error carries (A1 - A2)^2, which is O(1).  On a 12-site ring (J = 1,
    empty start, T = 1, coverage): the random schedule is first order, Lie is
    more accurate at the same step, and its advantage grows with q."""
    import scipy.sparse.linalg as spl
    N, prm, T = 12, (1.0, 1.0, 1.0, -0.5, 1.0), 1.0
    f = exact.observable_vectors("flip", N, 1)[:, 1] / N
    p0 = np.zeros(2 ** N)
    p0[0] = 1.0
    pe = spl.expm_multiply((exact.generator("flip", prm, N, 1, sparse=True).T * T).tocsr(), p0) @ f
    adv = []
    for q in (1, 2, 3, 6):
        cmap = np.array([i % 2 for i in range(N // q)], np.int32)
        At = [(exact.generator("flip", prm, N, 1, owner=exact.site_owner_by_colour(N, 1, q, 1, cmap, c),
                               sparse=True).T).tocsr() for c in range(2)]
        err_r, err_l = [], []
        for dt in (0.1, 0.05):
            cols, durs, _ = orc.schedule(_o.LIE, 2, dt, T)
            p = p0
            for c, d in zip(cols, durs):
                p = spl.expm_multiply(At[c] * d, p)
            err_l.append(abs(p @ f - pe))
            p = p0
            for _ in range(2 * int(round(T / dt))):
                p = 0.5 * (spl.expm_multiply(At[0] * dt, p) + spl.expm_multiply(At[1] * dt, p))
            err_r.append(abs(p @ f - pe))
        assert abs(err_r[0] / err_r[1] - 2.0) < 0.2, (q, err_r)
        assert err_l[0] < err_r[0] and err_l[1] < err_r[1], (q, err_l, err_r)
        adv.append(err_r[0] / err_l[0])
    assert all(b > a for a, b in zip(adv, adv[1:])), adv
