"""Pins for the oracle's nested (hierarchical) decomposition (Sec. 5, eqs.
sublatt2 and opdecomp2), independent of its code:

* window lists and colour maps of small cases, written out by hand from the
  definition (outer scheme, each outer window expanded into the inner one);
* the nested colourings pass the independence check (spin flip with 2 x 2
  colours, pair events with 4 x 4) and the pair models reject 2 x 2;
* with J = 0 every site operator commutes, so the nested scheme equals the
  outer scheme exactly for any inner step;
* as the inner step dtau -> 0 the nested propagator converges to the outer
  scheme's (with exact coarse-cell factors exp(d Q^c)), at first order for an
  inner Lie scheme and at second order for an inner Strang scheme -- exact
  matrix exponentials on a 4x2 lattice, no sampling;
* the blockwise oracle run with the nested list and map follows the nested
  split propagator (3 standard errors over replicas).
"""
import numpy as np
import pytest

import oracle as _o
from oracle import exact, nested
from _exact_stats import assert_within_3se, delta_state, moments

LIE, STRANG = _o.LIE, _o.STRANG


def test_window_lists_by_hand():
    c, d, e = nested.nested_schedule(LIE, 2, LIE, 2, 1.0, 0.5, 1.0)
    assert c.tolist() == [0, 1, 0, 1, 2, 3, 2, 3]
    assert d.tolist() == [0.5] * 8
    assert e.tolist() == [0] * 7 + [1]
    # outer Strang: (0, dt/2), (1, dt), (0, dt/2); inner Lie of step 0.5
    c, d, e = nested.nested_schedule(STRANG, 2, LIE, 2, 1.0, 0.5, 1.0)
    assert c.tolist() == [0, 1, 2, 3, 2, 3, 0, 1]
    assert d.tolist() == [0.5] * 8
    assert e.tolist() == [0] * 7 + [1]
    # inner Strang of step 0.5 inside outer Lie windows of 1.0, two outer steps
    c, d, e = nested.nested_schedule(LIE, 2, STRANG, 2, 1.0, 0.5, 2.0)
    one = [0, 1, 0, 0, 1, 0]
    assert c.tolist() == (one + [2, 3, 2, 2, 3, 2]) * 2
    assert d.tolist() == [0.25, 0.5, 0.25] * 8
    assert e.tolist() == ([0] * 11 + [1]) * 2
    # four outer colours, one inner colour: the outer scheme itself
    c, d, e = nested.nested_schedule(LIE, 4, LIE, 1, 0.2, 0.1, 0.2)
    assert c.tolist() == [0, 0, 1, 1, 2, 2, 3, 3] and d.tolist() == [0.1] * 8
    with pytest.raises(ValueError):  # 0.3 is not a whole number of inner steps of 0.2
        nested.nested_schedule(LIE, 2, LIE, 2, 0.3, 0.2, 0.3)
    with pytest.raises(ValueError):
        nested.nested_schedule(_o.RANDOM, 2, LIE, 2, 1.0, 0.5, 1.0)


def test_colour_maps_by_hand():
    cm = nested.nested_colour_map(8, 8, 1, 1, 2, 2, 2, 2).reshape(8, 8)
    assert cm[0].tolist() == [0, 1, 2, 3, 0, 1, 2, 3]
    assert cm[1].tolist() == [1, 0, 3, 2, 1, 0, 3, 2]
    assert cm[2].tolist() == [2, 3, 0, 1, 2, 3, 0, 1]
    assert cm[3].tolist() == [3, 2, 1, 0, 3, 2, 1, 0]
    # 4 x 4 colours on 2x2 coarse cells: outer (I%2)+2(J%2), inner (i%2)+2(j%2)
    cm = nested.nested_colour_map(8, 8, 2, 2, 2, 2, 4, 4).reshape(4, 4)
    assert cm[0].tolist() == [0, 1, 4, 5]
    assert cm[1].tolist() == [2, 3, 6, 7]
    assert cm[2].tolist() == [8, 9, 12, 13]
    assert cm[3].tolist() == [10, 11, 14, 15]
    with pytest.raises(ValueError):
        nested.nested_colour_map(12, 8, 2, 2, 4, 2, 2, 2)  # 6 block columns, coarse width 4


def test_nested_colourings_independent(orc):
    flip = orc.Model("flip", 16, 16)
    assert orc.decomp_check(flip, 2, 2, nested.nested_colour_map(16, 16, 2, 2, 2, 2, 2, 2), 4) == 0
    assert orc.decomp_check(flip, 2, 2, nested.nested_colour_map(16, 16, 2, 2, 4, 4, 2, 2), 4) == 0
    zgb = orc.Model("zgb", 16, 16)
    assert orc.decomp_check(zgb, 2, 2, nested.nested_colour_map(16, 16, 2, 2, 2, 2, 4, 4), 16) == 0
    assert orc.decomp_check(zgb, 2, 2, nested.nested_colour_map(16, 16, 2, 2, 2, 2, 2, 2), 4) != 0


# 4x2 lattice, 1x1 fine blocks, 2x1 coarse cells: a 2x2 grid of coarse cells,
# each with two fine blocks of different inner colour
LX, LY, CX, CY = 4, 2, 2, 1


def _generators(params, k_outer, k_inner):
    cm = nested.nested_colour_map(LX, LY, 1, 1, CX, CY, k_outer, k_inner)
    Qf = [exact.generator("flip", params, LX, LY, owner=exact.site_owner_by_colour(LX, LY, 1, 1, cm, c))
          for c in range(k_outer * k_inner)]
    Qo = [exact.generator("flip", params, LX, LY, owner=(cm // k_inner) == c) for c in range(k_outer)]
    return cm, Qf, Qo


def test_zero_coupling_nested_equals_outer(orc):
    params = (1.3, 0.7, 0.0, 0.0, 1.0)
    cm, Qf, Qo = _generators(params, 2, 2)
    assert orc.decomp_check(orc.Model("flip", LX, LY), 1, 1, cm, 4) == 0
    p0 = delta_state("flip", [1, 0, 0, 1, 1, 1, 0, 0])
    for osplit, isplit, dt, dtau in [(LIE, LIE, 0.5, 0.25), (STRANG, STRANG, 0.6, 0.1), (STRANG, LIE, 0.8, 0.4)]:
        oc, od, _ = _o.schedule(osplit, 2, dt, 2 * dt)
        c, d, _ = nested.nested_schedule(osplit, 2, isplit, 2, dt, dtau, 2 * dt)
        want = exact.split_propagate(p0, Qo, oc, od)
        got = exact.split_propagate(p0, Qf, c, d)
        assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("osplit,isplit,order", [(LIE, LIE, 1), (LIE, STRANG, 2), (STRANG, LIE, 1),
                                                 (STRANG, STRANG, 2)])
def test_inner_step_convergence_order(osplit, isplit, order):
    params = (1.0, 1.0, 1.5, 0.0, 1.0)
    _, Qf, Qo = _generators(params, 2, 2)
    p0 = delta_state("flip", [1, 1, 0, 0, 1, 0, 1, 0])
    dt, T = 0.4, 0.8
    oc, od, _ = _o.schedule(osplit, 2, dt, T)
    want = exact.split_propagate(p0, Qo, oc, od)
    errs = []
    for k in range(1, 5):
        dtau = 0.2 / 2 ** k  # divides dt and dt/2
        c, d, _ = nested.nested_schedule(osplit, 2, isplit, 2, dt, dtau, T)
        errs.append(np.abs(exact.split_propagate(p0, Qf, c, d) - want).sum())
    assert errs[-1] > 1e-9
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    lo, hi = (1.6, 2.5) if order == 1 else (3.2, 5.0)
    assert all(lo < r < hi for r in ratios[1:]), (errs, ratios)


def test_oracle_run_follows_nested_propagator(orc):
    params = (1.0, 1.0, 1.5, 0.0, 1.0)
    m = orc.Model("flip", LX, LY, k_a=1.0, k_d=1.0, J=1.5, h=0.0, beta=1.0)
    cm, Qf, _ = _generators(params, 2, 2)
    lat0 = np.array([1, 1, 0, 0, 1, 0, 1, 0], np.uint8)
    cols, durs, ends = nested.nested_schedule(LIE, 2, STRANG, 2, 0.5, 0.25, 1.0)
    R = 3000
    sample = np.array([orc.fs_run(m, lat0, 1, 1, cm, 4, cols, durs, 0, r, observe_flags=ends)["obs"]
                       for r in range(R)], dtype=np.float64)
    ov = exact.observable_vectors("flip", LX, LY)
    p = delta_state("flip", lat0)
    start = 0
    for k, w_end in enumerate(np.nonzero(ends)[0]):
        p = exact.split_propagate(p, Qf, cols[start:w_end + 1], durs[start:w_end + 1])
        start = w_end + 1
        mean, var = moments(p, ov)
        assert_within_3se(sample[:, k, :], mean, var, (1, 4), label=("nested", k))
