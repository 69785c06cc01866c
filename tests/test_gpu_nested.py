"""Parity of the nested (hierarchical) sweep with the CPU oracle (needs a GPU).

A nested sim runs one launch per outer window: one workgroup per coarse cell,
its fine blocks one wave each on a shared LDS tile, the inner windows
separated by workgroup barriers.  The oracle builds the nested window list and
colour map on its own (oracle/nested.py) and runs them through its blockwise
fractional-step scheme.  Compared bit for bit at every outer-window boundary:
the lattice, and W of every block active in the last inner window.  The same
runs with the nested kernel switched off (flat sweeps on the same list) give
the same bits.
"""
import numpy as np
import pytest

from oracle import nested

pytestmark = pytest.mark.gpu

LIE, STRANG = 0, 1


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


@pytest.fixture(scope="module")
def ctx(F):
    c = F.fskmc_ctx_create(0)
    yield c
    F.fskmc_ctx_destroy(c)


def _model(orc, kind, L, params):
    if kind == "flip":
        k_a, k_d, J, h, beta = params
        return orc.Model(kind, L, L, k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    if kind == "kawasaki":
        D, J, beta = params
        return orc.Model(kind, L, L, D=D, J=J, beta=beta)
    y, k_r, D = params
    return orc.Model(kind, L, L, y=y, k_r=k_r, D=D)


CASES = {
    # kind, L, params, b, c, k_outer, k_inner, outer split, inner split, dt, dtau, T, init
    "flip256-b16-c4-lie-lie": ("flip", 256, (1.0, 1.0, 1.0, 0.0, 1.0), 16, 4, 2, 2, LIE, LIE, 0.2, 0.1, 2.0,
                               "bernoulli"),
    "flip256-b8-c2-strang-strang": ("flip", 256, (1.0, 1.0, 1.5, -0.3, 1.0), 8, 2, 2, 2, STRANG, STRANG, 0.4,
                                    0.1, 2.0, "bernoulli"),
    "flip256-b32-c4-k4x4-lie-strang": ("flip", 256, (1.0, 1.0, 0.5, 0.2, 1.0), 32, 4, 4, 4, LIE, STRANG, 0.5,
                                       0.25, 2.0, "empty"),
    "reaction256-b16-c4": ("zgb", 256, (0.5, 1000.0, 10.0), 16, 4, 4, 4, STRANG, LIE, 0.05, 0.025, 0.5, "empty"),
    "kawasaki256-b16-c2": ("kawasaki", 256, (4.0, 1.0, 1.0), 16, 2, 4, 4, LIE, STRANG, 0.5, 0.25, 3.0,
                           "bernoulli"),
    "flip1024-b16-c4-full-size": ("flip", 1024, (1.0, 1.0, 1.0, 0.0, 1.0), 16, 4, 2, 2, LIE, LIE, 0.1, 0.05, 0.3,
                                  "bernoulli"),
    "flip1024-b16-c2-full-size": ("flip", 1024, (1.0, 1.0, 1.5, 0.0, 1.0), 16, 2, 2, 2, STRANG, LIE, 0.2, 0.05,
                                  0.4, "bernoulli"),
}
FLIP_CASES = sorted(k for k in CASES if k.startswith("flip"))


def _run_case(F, orc, ctx, name, kernel_on, cx=None):
    kind, L, prm, b, c, ko, ki, osp, isp, dt, dtau, T, init = CASES[name]
    cx = c if cx is None else cx
    cy = c
    F.fskmc_ctx_set_nested(ctx, kernel_on)
    sim = F.Sim(ctx, kind, L, L, prm, bx=b, by=b, dt=dt, T=T, split=osp, seed=1, replica=5,
                nested=dict(cx=cx, cy=cy, outer_colours=ko, inner_colours=ki, inner_split=isp, dtau=dtau))
    model = _model(orc, kind, L, prm)
    cmap = nested.nested_colour_map(L, L, b, b, cx, cy, ko, ki)
    if L <= 256:  # the oracle's checker is quadratic in the blocks; larger maps repeat the same pattern
        assert orc.decomp_check(model, b, b, cmap, ko * ki) == 0
    cols, durs, ends = nested.nested_schedule(osp, ko, isp, ki, dt, dtau, T)
    assert sim.windows() == (len(cols), 0)
    if init == "bernoulli":
        sim.init(1, 0.5)
        lat = orc.init_bernoulli(L * L, 0.5, 1, 5)
    else:
        sim.init(0)
        lat = np.zeros(L * L, np.uint8)
    n0 = int(lat.sum())
    # outer-window boundaries: a new outer window starts where the outer colour changes
    # or an inner scheme restarts; the oracle list is cut where the library cuts it
    outer = [w for w in range(len(cols)) if w == 0 or cols[w] // ki != cols[w - 1] // ki or ends[w - 1]]
    per_outer = {}
    for w in range(len(cols)):
        per_outer.setdefault(max(o for o in outer if o <= w), []).append(w)
    res = orc.fs_run(model, lat, b, b, cmap, ko * ki, cols, durs, 1, 5, want_W=True,
                     want_snap=L * L * len(cols) <= (1 << 26))
    events = 0
    snaps = res.get("snap")
    for start in outer:
        ws = per_outer[start]
        sim.advance(len(ws))
        last = ws[-1]
        W = sim.block_events()
        active = cmap == cols[last]
        np.testing.assert_array_equal(W[active], res["W"][last][active])
        events += int(res["W"][ws].sum())
        if snaps is not None:
            got = sim.lattice()
            assert np.array_equal(got, snaps[last]), (name, last, int((got != snaps[last]).sum()))
    got = sim.lattice()
    assert np.array_equal(got, res["lattice"]), int((got != res["lattice"]).sum())
    obs = sim.observe()
    assert obs["events"] == res["events"] == events and events > 0
    if kind == "kawasaki":
        assert obs["count"][1] == n0
    sim.close()
    F.fskmc_ctx_set_nested(ctx, 1)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("kernel_on", [1, 0], ids=["nested-kernel", "flat-sweeps"])
def test_nested_matches_oracle(F, orc, ctx, name, kernel_on):
    _run_case(F, orc, ctx, name, kernel_on)


def test_nested_rectangular_cells_use_flat_sweeps(F, orc, ctx):
    """Cells of 2 x 4 blocks have no nested kernel variant: the flat sweeps
    run the same list and still give the oracle's bits."""
    _run_case(F, orc, ctx, "flip256-b16-c4-lie-lie", 1, cx=2)


@pytest.mark.parametrize("resident", [1, 0], ids=["resident", "per-outer-window"])
def test_nested_persistent_setting_outer_window_calls(F, orc, ctx, resident):
    """With the persistent setting a spin-flip nested sim advanced one outer
    window per call runs resident launches (resident knob on) or one launch
    per outer window (off); both give the oracle's bits at every call."""
    F.fskmc_ctx_set_persistent(ctx, 50)
    F.fskmc_ctx_set_resident(ctx, resident)
    try:
        _run_case(F, orc, ctx, "flip256-b8-c2-strang-strang", 1)
    finally:
        F.fskmc_ctx_set_persistent(ctx, 0)
        F.fskmc_ctx_set_resident(ctx, 1)


def test_nested_invalid(F, ctx):
    E = F.FskmcError

    def make(kind="flip", L=256, prm=(1.0, 1.0, 1.0, 0.0, 1.0), b=16, split=LIE, dt=0.2, T=1.0, **kw):
        n = dict(cx=4, cy=4, outer_colours=2, inner_colours=2, inner_split=LIE, dtau=0.1)
        n.update(kw)
        return F.Sim(ctx, kind, L, L, prm, bx=b, by=b, dt=dt, T=T, split=split, nested=n)

    for kw, code in [(dict(outer_colours=2, inner_colours=4), None),
                     (dict(dtau=0.15), F.FSKMC_EINVAL),          # 0.2 is not a whole number of 0.15 steps
                     (dict(inner_colours=3), F.FSKMC_EINVAL),
                     (dict(inner_split=2), F.FSKMC_EINVAL),      # random inner scheme
                     (dict(split=2), F.FSKMC_EINVAL),            # random outer scheme
                     (dict(cx=3), F.FSKMC_EINVAL),               # 16 block columns, cells of 3
                     (dict(L=64), F.FSKMC_EDECOMP),              # one coarse cell per row
                     ]:
        if code is None:
            make(**kw).close()
            continue
        with pytest.raises(E) as ei:
            make(**kw)
        assert ei.value.code == code, kw
    with pytest.raises(E) as ei:  # pair events with 2 outer colours: diagonal cells share a ring site
        make(kind="zgb", prm=(0.5, 1000.0, 10.0), outer_colours=2, inner_colours=4)
    assert ei.value.code == F.FSKMC_EDECOMP
    with pytest.raises(E) as ei:  # pair events with 2 inner colours
        make(kind="zgb", prm=(0.5, 1000.0, 10.0), outer_colours=4, inner_colours=2)
    assert ei.value.code == F.FSKMC_EDECOMP


@pytest.mark.parametrize("name", FLIP_CASES)
@pytest.mark.parametrize("persist", [100000, 7], ids=["whole-run", "7-windows-per-launch"])
def test_nested_resident_matches_oracle(F, orc, ctx, name, persist):
    """Spin-flip nested sims with persistent launches: every coarse cell is a
    workgroup resident for the whole launch, cells exchange tagged boundary
    words between outer windows.  Advanced 11 windows per call, so launches
    also start and end inside outer windows; the final lattice, the events and
    W of the last window's active blocks equal the oracle's."""
    kind, L, prm, b, c, ko, ki, osp, isp, dt, dtau, T, init = CASES[name]
    F.fskmc_ctx_set_persistent(ctx, persist)
    F.fskmc_ctx_set_resident(ctx, 1)
    try:
        sim = F.Sim(ctx, kind, L, L, prm, bx=b, by=b, dt=dt, T=T, split=osp, seed=1, replica=9,
                    nested=dict(cx=c, cy=c, outer_colours=ko, inner_colours=ki, inner_split=isp, dtau=dtau))
        model = _model(orc, kind, L, prm)
        cmap = nested.nested_colour_map(L, L, b, b, c, c, ko, ki)
        cols, durs, ends = nested.nested_schedule(osp, ko, isp, ki, dt, dtau, T)
        if init == "bernoulli":
            sim.init(1, 0.5)
            lat = orc.init_bernoulli(L * L, 0.5, 1, 9)
        else:
            sim.init(0)
            lat = np.zeros(L * L, np.uint8)
        res = orc.fs_run(model, lat, b, b, cmap, ko * ki, cols, durs, 1, 9, want_W=True)
        while sim.windows()[1] < sim.windows()[0]:
            sim.advance(min(11, sim.windows()[0] - sim.windows()[1]))
        F.fskmc_sync(ctx)
        got = sim.lattice()
        assert np.array_equal(got, res["lattice"]), int((got != res["lattice"]).sum())
        assert sim.observe()["events"] == res["events"] > 0
        active = cmap == cols[-1]
        np.testing.assert_array_equal(sim.block_events()[active], res["W"][-1][active])
        sim.close()
    finally:
        F.fskmc_ctx_set_persistent(ctx, 0)


def test_nested_resident_wait_timeout_reports_edevice(F, orc, ctx):
    """A wait limit of one clock tick makes the cells' bounded waits give up:
    the launch aborts, the next synchronising call reports FSKMC_EDEVICE, and
    a fresh sim on the same context then matches the oracle again."""
    F.fskmc_ctx_set_persistent(ctx, 100000)
    F.fskmc_ctx_set_resident(ctx, 1)
    try:
        sim = F.Sim(ctx, "flip", 256, 256, (1.0, 1.0, 1.0, 0.0, 1.0), bx=16, by=16, dt=0.2, T=4.0, split=LIE,
                    nested=dict(cx=2, cy=2, outer_colours=2, inner_colours=2, inner_split=LIE, dtau=0.1))
        sim.init(1, 0.5)
        F.fskmc_ctx_set_wait_limit(ctx, 1e-8)
        sim.run_to_end()
        with pytest.raises(F.FskmcError) as ei:
            F.fskmc_sync(ctx)
        assert ei.value.code == F.FSKMC_EDEVICE
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        sim.close()
    finally:
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        F.fskmc_ctx_set_persistent(ctx, 0)
    _run_case(F, orc, ctx, "flip256-b8-c2-strang-strang", 1)
