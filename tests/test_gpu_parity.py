"""Parity of the HIP fractional-step sweep with the CPU oracle (needs a GPU).

Bit-exact: the lattice after every window (small cases) or after sampled
windows (full-size cases), the per-block event counts W of every active block,
the host-built rate tables, the Bernoulli initial state and the integer
observables.  Every call goes through the C ABI of libfskmc.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FLIP = "flip"
ZGB = "zgb"
KAW = "kawasaki"


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


@pytest.fixture(scope="module")
def ctx(F):
    c = F.fskmc_ctx_create(0)
    yield c
    F.fskmc_ctx_destroy(c)


def _orc_model(orc, kind, Lx, Ly, params):
    if kind == FLIP:
        k_a, k_d, J, h, beta = params
        return orc.Model(FLIP, Lx, Ly, k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    if kind == KAW:
        D, J, beta = params
        return orc.Model(KAW, Lx, Ly, D=D, J=J, beta=beta)
    y, k_r, D = params
    return orc.Model(ZGB, Lx, Ly, y=y, k_r=k_r, D=D)


def _split_code(name):
    return {"lie": 0, "strang": 1, "random": 2}[name]


class Pair:
    """A GPU simulation and its oracle twin on the same inputs."""

    def __init__(self, F, orc, ctx, kind, Lx, Ly, params, b, ncol, dt, T, split, seed=0, replica=0,
                 init="empty", lattice0=None, colour_map=None):
        self.F, self.orc = F, orc
        self.kind = kind
        dim = 1 if Ly == 1 else 2
        self.bx, self.by = (b, b) if dim == 2 else (b, 1)
        self.sim = F.Sim(ctx, kind, Lx, Ly, params, bx=self.bx, by=self.by, n_colours=ncol, dt=dt, T=T,
                         split=_split_code(split), seed=seed, replica=replica, colour_map=colour_map)
        self.model = _orc_model(orc, kind, Lx, Ly, params)
        self.N = Lx * Ly
        self.seed, self.replica, self.ncol = seed, replica, ncol
        self.cmap = (np.asarray(colour_map, np.int32) if colour_map is not None
                     else orc.colour_map(self.model, self.bx, self.by, ncol))
        self.cols, self.durs, self.ends = orc.schedule(_split_code(split), ncol, dt, T, seed, replica)
        if init == "empty":
            self.sim.init(0)
            self.lat = np.zeros(self.N, np.uint8)
        elif init == "bernoulli":
            self.sim.init(1, 0.5)
            self.lat = orc.init_bernoulli(self.N, 0.5, seed, replica)
        else:
            self.lat = np.asarray(lattice0, np.uint8).ravel().copy()
            self.sim.set_lattice(self.lat)
        self.w = 0

    def step_compare_each(self, n):
        """Advance n windows one by one; compare the lattice and W each time."""
        res = self.orc.fs_run(self.model, self.lat, self.bx, self.by, self.cmap, self.ncol,
                              self.cols[self.w:self.w + n], self.durs[self.w:self.w + n], self.seed,
                              self.replica, w0=self.w, want_W=True, want_snap=True)
        events = 0
        for i in range(n):
            self.sim.advance(1)
            got = self.sim.lattice()
            want = res["snap"][i]
            assert np.array_equal(got, want), (self.w + i, int((got != want).sum()))
            active = self.cmap == self.cols[self.w + i]
            W = self.sim.block_events()
            np.testing.assert_array_equal(W[active], res["W"][i][active])
            events += int(res["W"][i].sum())
        self.lat = res["lattice"]
        self.w += n
        return events

    def step_compare_end(self, n):
        """Advance n windows in one call; compare the final lattice and events."""
        res = self.orc.fs_run(self.model, self.lat, self.bx, self.by, self.cmap, self.ncol,
                              self.cols[self.w:self.w + n], self.durs[self.w:self.w + n], self.seed,
                              self.replica, w0=self.w, want_W=True)
        self.sim.advance(n)
        got = self.sim.lattice()
        assert np.array_equal(got, res["lattice"]), int((got != res["lattice"]).sum())
        W = self.sim.block_events()
        last = self.cols[self.w + n - 1]
        active = self.cmap == last
        np.testing.assert_array_equal(W[active], res["W"][n - 1][active])
        self.lat = res["lattice"]
        self.w += n
        return res["events"]


def test_rate_tables_bitwise(F, orc, ctx):
    cases = [(FLIP, 64, 64, (1.0, 1.0, 1.0, 0.0, 1.0), 8, 2), (FLIP, 256, 1, (0.3, 2.5, 2.0, -1.0, 1.7), 64, 2),
             (FLIP, 64, 64, (1.0, 1.0, 0.5, 0.3, 3.0), 16, 2), (ZGB, 64, 64, (0.53, 1000.0, 10.0), 32, 4),
             (ZGB, 64, 64, (0.3, 7.5, 0.0), 16, 4), (KAW, 64, 64, (4.0, 1.0, 1.0), 16, 4),
             (KAW, 64, 64, (1.0, -0.7, 2.0), 32, 4), (KAW, 64, 64, (0.0, 0.0, 1.0), 8, 4)]
    for kind, Lx, Ly, prm, b, ncol in cases:
        p = Pair(F, orc, ctx, kind, Lx, Ly, prm, b, ncol, 0.1, 0.2, "lie")
        got = p.sim.rate_table()
        want = orc.rate_table(p.model)
        assert got.tobytes() == want.tobytes(), kind
        p.sim.close()


def test_bernoulli_init_bitwise(F, orc, ctx):
    for (Lx, Ly, seed, rep) in [(64, 64, 0, 0), (1024, 1024, 0, 3), (512, 1, 7, 11)]:
        s = F.Sim(ctx, FLIP, Lx, Ly, (1, 1, 1, 0, 1), b=8 if Ly > 1 else 64, dt=0.1, T=0.1, seed=seed, replica=rep)
        s.init(1, 0.5)
        np.testing.assert_array_equal(s.lattice(), orc.init_bernoulli(Lx * Ly, 0.5, seed, rep))
        s.init(1, 0.3)
        np.testing.assert_array_equal(s.lattice(), orc.init_bernoulli(Lx * Ly, 0.3, seed, rep))
        s.close()


def test_config0_every_window(F, orc, ctx):
    """64x64, J=1, 8x8 blocks, 2 colours, Lie dt=0.1, T=10, empty start, seed 0:
    the whole run, lattice and block counts after every window."""
    p = Pair(F, orc, ctx, FLIP, 64, 64, (1.0, 1.0, 1.0, 0.0, 1.0), 8, 2, 0.1, 10.0, "lie")
    total, nxt = p.sim.windows()
    assert total == 200 and nxt == 0
    ev = p.step_compare_each(200)
    obs = p.sim.observe()
    want = orc.observe(p.model, p.lat)
    assert obs["count"][:2] == list(want[:2]) and obs["bonds_equal"][1] == want[4]
    assert obs["events"] == ev and obs["window"] == 200 and obs["steps"] == 100
    assert abs(obs["t"] - 10.0) < 1e-12
    with pytest.raises(F.FskmcError):
        p.sim.advance(1)


@pytest.mark.parametrize("wpg", [1, 2, 4, 8])
def test_waves_per_group_is_result_neutral(F, orc, ctx, wpg):
    F.fskmc_ctx_set_waves_per_group(ctx, wpg)
    try:
        p = Pair(F, orc, ctx, FLIP, 128, 128, (1.0, 1.0, 0.5, 0.0, 1.0), 16, 2, 0.5, 5.0, "strang",
                 init="bernoulli", seed=3, replica=1)
        p.step_compare_end(15)
    finally:
        F.fskmc_ctx_set_waves_per_group(ctx, 2)


@pytest.mark.parametrize("J,dt,split", [(0.5, 1.0, "lie"), (1.0, 0.1, "lie"), (2.0, 0.1, "strang"),
                                        (1.0, 0.01, "strang"), (0.5, 1.0, "random")])
def test_config1_shape_small(F, orc, ctx, J, dt, split):
    """The 16x16-block Ising sweep of the 1024^2 workload on a 256^2 lattice,
    every window, several (J, dt, split)."""
    p = Pair(F, orc, ctx, FLIP, 256, 256, (1.0, 1.0, J, 0.0, 1.0), 16, 2, dt, 100.0, split, init="bernoulli",
             seed=0, replica=5)
    p.step_compare_each(12)


def test_config1_full_size_sampled(F, orc, ctx):
    """1024^2, J=1, Lie dt=0.1 from Bernoulli(1/2): every window of the first
    step compared, then batches of windows compared at their ends."""
    p = Pair(F, orc, ctx, FLIP, 1024, 1024, (1.0, 1.0, 1.0, 0.0, 1.0), 16, 2, 0.1, 100.0, "lie",
             init="bernoulli", seed=0, replica=0)
    p.step_compare_each(2)
    p.step_compare_end(6)


def test_config1_full_size_long_window(F, orc, ctx):
    """1024^2, J=0.5, dt=1 (about 80 events per block-window)."""
    p = Pair(F, orc, ctx, FLIP, 1024, 1024, (1.0, 1.0, 0.5, 0.0, 1.0), 16, 2, 1.0, 100.0, "lie",
             init="bernoulli", seed=0, replica=2)
    p.step_compare_each(2)


@pytest.mark.parametrize("b", [8, 16, 32])
def test_flip_block_sizes(F, orc, ctx, b):
    p = Pair(F, orc, ctx, FLIP, 4 * b * 2, 2 * b * 2, (0.7, 1.3, 1.2, -0.4, 1.1), b, 2, 0.4, 4.0, "strang",
             init="bernoulli", seed=9, replica=b)
    p.step_compare_each(9)


@pytest.mark.parametrize("Lx,Ly,b", [(2112, 2048, 32), (4100 * 1024, 1, 1024)], ids=["2d-32x32", "1d-1024"])
def test_sixteen_sites_per_lane_full_launch(F, orc, ctx, Lx, Ly, b):
    """More than 2048 active blocks of 16 sites per lane (2112 and 2050 per
    colour): launches that big take the full-launch kernel, whose descent hands
    the chosen lane's leaves over through LDS, not the small-launch kernel the
    smaller cases take; three windows compared in full."""
    p = Pair(F, orc, ctx, FLIP, Lx, Ly, (1.0, 1.0, 0.8, -0.2, 1.0), b, 2, 0.2, 5.0, "lie", init="bernoulli", seed=5,
             replica=b)
    p.step_compare_each(3)


@pytest.mark.parametrize("b", [64, 256, 1024])
def test_flip_1d_rows(F, orc, ctx, b):
    p = Pair(F, orc, ctx, FLIP, 8 * b, 1, (1.0, 1.0, 1.0, -0.5, 1.0), b, 2, 1.0, 10.0, "lie", init="bernoulli",
             seed=1, replica=b)
    p.step_compare_each(8)


@pytest.mark.parametrize("y,D,split", [(0.5, 10.0, "strang"), (0.53, 0.0, "strang"), (0.3, 10.0, "lie")])
def test_reaction_model_4_colours(F, orc, ctx, y, D, split):
    """3-state A/B reaction model, 32x32 blocks, 4 colours, pair events that
    write into the halo, stiff k_r = 1e3."""
    p = Pair(F, orc, ctx, ZGB, 256, 256, (y, 1000.0, D), 32, 4, 0.05, 10.0, split, seed=0, replica=1)
    p.step_compare_each(14)
    p.step_compare_end(14)
    obs = p.sim.observe()
    want = orc.observe(p.model, p.lat)
    assert obs["count"] == list(want[:3]) and obs["bonds_equal"] == list(want[3:6]) and obs["bonds_ab"] == want[6]


@pytest.mark.parametrize("b", [8, 16])
def test_reaction_model_small_blocks(F, orc, ctx, b):
    p = Pair(F, orc, ctx, ZGB, 128, 128, (0.45, 40.0, 3.0), b, 4, 0.1, 2.0, "strang", seed=4, replica=b)
    p.step_compare_each(14)


@pytest.mark.parametrize("D,J,split,b", [(4.0, 1.0, "strang", 32), (4.0, -0.5, "lie", 16), (2.0, 2.0, "random", 8),
                                         (4.0, 0.0, "strang", 32)],
                         ids=["repulsive-strang-b32", "attractive-lie-b16", "random-b8", "exclusion-b32"])
def test_kawasaki_every_window(F, orc, ctx, D, J, split, b):
    """Conserved spin exchange: particles hop into the halo of the block, 4
    colours; every window bit-exact, the particle number invariant."""
    p = Pair(F, orc, ctx, KAW, 256, 256, (D, J, 1.0), b, 4, 0.25, 20.0, split, init="bernoulli", seed=2, replica=b)
    n0 = int(p.lat.sum())
    assert p.step_compare_each(14) > 0
    p.step_compare_end(14)
    obs = p.sim.observe()
    want = orc.observe(p.model, p.lat)
    assert obs["count"][1] == n0 and obs["count"][2] == 0
    assert obs["count"] == list(want[:3]) and obs["bonds_equal"] == list(want[3:6])


def test_kawasaki_full_size_first_windows(F, orc, ctx):
    """4096^2 half-filled exchange lattice, 32x32 blocks, Strang: the first
    two windows compared in full."""
    p = Pair(F, orc, ctx, KAW, 4096, 4096, (4.0, 1.0, 1.0), 32, 4, 0.05, 10.0, "strang", init="bernoulli",
             seed=0, replica=0)
    p.step_compare_each(2)


def test_config2_full_size_first_windows(F, orc, ctx):
    """4096^2 reaction lattice, 32x32 blocks, Strang dt=0.05: the first two
    windows compared in full."""
    p = Pair(F, orc, ctx, ZGB, 4096, 4096, (0.5, 1000.0, 10.0), 32, 4, 0.05, 10.0, "strang", seed=0, replica=0)
    p.step_compare_each(2)


def test_edge_zero_total_rate(F, orc, ctx):
    """Blocks whose total rate is zero draw nothing: an all-B reaction lattice
    and an empty lattice without adsorption."""
    p = Pair(F, orc, ctx, ZGB, 64, 64, (0.5, 1000.0, 10.0), 16, 4, 0.1, 1.0, "lie", init="given",
             lattice0=np.full(64 * 64, 2, np.uint8))
    p.step_compare_each(4)
    assert np.all(p.sim.block_events() == 0)
    q = Pair(F, orc, ctx, FLIP, 64, 64, (0.0, 1.0, 1.0, 0.0, 1.0), 8, 2, 0.1, 1.0, "lie")
    q.step_compare_each(4)
    assert q.sim.observe()["events"] == 0


def test_edge_ragged_custom_colouring(F, orc, ctx):
    """A 3-colour map with unequal colour classes on a 1D ring (NBX = 10):
    colours 0 and 1 have four blocks, colour 2 has two."""
    cmap = np.array([0, 1, 2, 0, 1, 2, 0, 1, 0, 1], np.int32)
    assert orc.decomp_check(orc.Model(FLIP, 640, 1), 64, 1, cmap, 3) == 0
    p = Pair(F, orc, ctx, FLIP, 640, 1, (1.0, 1.0, 1.0, 0.0, 1.0), 64, 3, 0.5, 5.0, "strang", init="bernoulli",
             colour_map=cmap)
    p.step_compare_each(25)


def test_edge_invalid_inputs(F, ctx):
    E = F.FskmcError
    with pytest.raises(E) as ei:  # pair events with a 2-colour checkerboard
        F.Sim(ctx, ZGB, 64, 64, (0.5, 1000.0, 0.0), b=16, n_colours=2, dt=0.1, T=1.0)
    assert ei.value.code == F.FSKMC_EDECOMP
    with pytest.raises(E):  # T/dt not an integer
        F.Sim(ctx, FLIP, 64, 64, (1, 1, 1, 0, 1), b=8, dt=0.3, T=1.0)
    with pytest.raises(E) as ei:  # 3e9 windows: beyond the device's 32-bit window indices, rejected before allocating
        F.Sim(ctx, FLIP, 64, 64, (1, 1, 1, 0, 1), b=8, dt=1e-9, T=3.0)
    assert ei.value.code == F.FSKMC_EINVAL
    with pytest.raises(E):  # unsupported block
        F.Sim(ctx, FLIP, 60, 60, (1, 1, 1, 0, 1), b=12, dt=0.1, T=1.0)
    with pytest.raises(E):  # odd number of blocks breaks the 2-colour checkerboard
        F.Sim(ctx, FLIP, 24, 24, (1, 1, 1, 0, 1), b=8, dt=0.1, T=1.0)
    with pytest.raises(E) as ei:  # spin exchange is a pair model: no 2-colour checkerboard
        F.Sim(ctx, KAW, 64, 64, (1.0, 1.0, 1.0), b=16, n_colours=2, dt=0.1, T=1.0)
    assert ei.value.code == F.FSKMC_EDECOMP
    with pytest.raises(E) as ei:  # pair models are two-dimensional
        F.Sim(ctx, KAW, 1024, 1, (1.0, 1.0, 1.0), b=64, n_colours=2, dt=0.1, T=1.0)
    assert ei.value.code == F.FSKMC_EINVAL
    for bad in ((-1.0, 1.0, 1.0), (1.0, float("inf"), 1.0), (1.0, 1.0, float("nan"))):
        with pytest.raises(E) as ei:
            F.Sim(ctx, KAW, 64, 64, bad, b=16, n_colours=4, dt=0.1, T=1.0)
        assert ei.value.code == F.FSKMC_EINVAL
    k = F.Sim(ctx, KAW, 64, 64, (1.0, 1.0, 1.0), b=16, n_colours=4, dt=0.1, T=0.1)
    with pytest.raises(E):  # exchange has states {0, 1} only
        k.set_lattice(np.full(4096, 2, np.uint8))
    k.close()
    s = F.Sim(ctx, FLIP, 64, 64, (1, 1, 1, 0, 1), b=8, dt=0.1, T=0.1)
    with pytest.raises(E):  # state outside the spin space
        s.set_lattice(np.full(4096, 2, np.uint8))
    s.close()
    for bad in (0.0, -1.0, 61.0, float("nan")):  # wait limit outside (0, 60] s
        with pytest.raises(E) as ei:
            F.fskmc_ctx_set_wait_limit(ctx, bad)
        assert ei.value.code == F.FSKMC_EINVAL
    with pytest.raises(E) as ei:  # negative windows per persistent launch
        F.fskmc_ctx_set_persistent(ctx, -1)
    assert ei.value.code == F.FSKMC_EINVAL


def test_edge_zero_length_schedule(F, ctx):
    s = F.Sim(ctx, FLIP, 64, 64, (1, 1, 1, 0, 1), b=8, dt=0.1, T=0.0)
    assert s.windows() == (0, 0)
    s.run_to_end()
    assert s.observe()["count"][0] == 4096
    s.close()


def test_checkpoint_resume_bitwise(F, orc, ctx):
    kw = dict(kind=FLIP, Lx=256, Ly=256, params=(1.0, 1.0, 0.7, 0.1, 1.0), b=16, n_colours=2, dt=0.2, T=4.0,
              split=F.FSKMC_STRANG, seed=2, replica=4)
    a = F.Sim(ctx, **kw)
    a.init(1, 0.5)
    a.advance(17)
    w, lat = a.get_state()
    assert w == 17
    a.run_to_end()
    b = F.Sim(ctx, **kw)
    b.set_state(w, lat)
    b.run_to_end()
    np.testing.assert_array_equal(a.lattice(), b.lattice())
    a.close()
    b.close()


def test_attach_torch_lattice(F, orc, ctx):
    import torch
    t = torch.zeros(128 * 128, dtype=torch.uint8, device="cuda")
    s = F.Sim(ctx, FLIP, 128, 128, (1.0, 1.0, 1.0, 0.0, 1.0), b=16, dt=0.1, T=1.0, seed=0, replica=8)
    F.fskmc_sim_attach_device_lattice(s.handle, t.data_ptr(), t.numel())
    s.init(1, 0.5)
    s.run_to_end()
    F.fskmc_sync(ctx)
    model = orc.Model(FLIP, 128, 128, J=1.0)
    cols, durs, _ = orc.schedule(0, 2, 0.1, 1.0)
    res = orc.fs_run(model, orc.init_bernoulli(128 * 128, 0.5, 0, 8), 16, 16, orc.colour_map(model, 16, 16, 2), 2,
                     cols, durs, 0, 8)
    np.testing.assert_array_equal(t.cpu().numpy(), res["lattice"])
    s.close()


def test_batch_equals_alone(F, orc, ctx):
    """Sims of different sizes, models and schedules advanced together in one
    batched launch per window give the same bits as each advanced alone."""
    specs = [
        dict(kind=FLIP, Lx=128, Ly=128, params=(1.0, 1.0, 1.5, -0.5, 1.0), b=16, n_colours=2, dt=0.1, T=2.0,
             split=0, seed=0, replica=1),
        dict(kind=FLIP, Lx=256, Ly=256, params=(1.0, 1.0, 0.3, 0.8, 1.0), b=16, n_colours=2, dt=0.2, T=2.0,
             split=1, seed=0, replica=2),
        dict(kind=FLIP, Lx=64, Ly=64, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=8, n_colours=2, dt=0.1, T=10.0,
             split=0, seed=0, replica=3),
        dict(kind=ZGB, Lx=128, Ly=128, params=(0.5, 1000.0, 10.0), b=32, n_colours=4, dt=0.05, T=1.0, split=1,
             seed=0, replica=4),
        dict(kind=FLIP, Lx=512, Ly=1, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=64, n_colours=2, dt=1.0, T=5.0,
             split=0, seed=0, replica=5),
        dict(kind=KAW, Lx=128, Ly=128, params=(4.0, 1.0, 1.0), b=32, n_colours=4, dt=0.25, T=3.0, split=1,
             seed=0, replica=6),
    ]
    alone, batch = [], []
    for sp in specs:
        a = F.Sim(ctx, **sp)
        b = F.Sim(ctx, **sp)
        a.init(1, 0.5)
        b.init(1, 0.5)
        a.run_to_end()
        alone.append(a)
        batch.append(b)
    handles = [b.handle for b in batch]
    while any(b.windows()[1] < b.windows()[0] for b in batch):
        F.fskmc_batch_advance(ctx, handles, 7)
    for a, b in zip(alone, batch):
        np.testing.assert_array_equal(a.lattice(), b.lattice())
        assert a.observe()["events"] == b.observe()["events"]
        a.close()
        b.close()


@pytest.mark.parametrize("case", [
    (FLIP, 64, 64, (1.0, 1.0, 1.0, 0.0, 1.0), 8, 2, 0.1, 10.0, "lie", "empty", 7),
    (FLIP, 256, 256, (1.0, 1.0, 0.5, 0.2, 1.0), 16, 2, 0.1, 100.0, "strang", "bernoulli", 16),
    (FLIP, 256, 256, (1.0, 1.0, 2.0, -0.3, 1.0), 32, 2, 1.0, 100.0, "random", "bernoulli", 5),
    (FLIP, 4096, 1, (1.0, 1.0, 1.0, -0.5, 1.0), 256, 2, 1.0, 100.0, "lie", "bernoulli", 9),
    (ZGB, 256, 256, (0.5, 1000.0, 10.0), 32, 4, 0.05, 10.0, "strang", "empty", 11),
    (FLIP, 16, 16, (1.0, 1.0, 1.0, 0.2, 1.0), 8, 2, 0.5, 20.0, "strang", "bernoulli", 6),
    (FLIP, 128, 1, (1.0, 1.0, 1.5, 0.0, 1.0), 64, 2, 1.0, 50.0, "random", "bernoulli", 13),
    (KAW, 256, 256, (4.0, 1.0, 1.0), 32, 4, 0.25, 20.0, "strang", "bernoulli", 9),
], ids=["flip64-b8", "flip256-b16-strang", "flip256-b32-random", "flip1d-b256", "zgb256-b32", "flip16-b8-2x2",
        "flip1d-128-b64-two-blocks", "kawasaki256-b32"])
@pytest.mark.parametrize("resident", [1, 0], ids=["resident", "streaming"])
def test_persistent_sweep_bitwise(F, orc, ctx, case, resident):
    """Several windows inside one persistent kernel (neighbour-only waits
    instead of a launch per window) give the oracle's bits, with the blocks
    kept in LDS across windows (spin flip) or streamed from HBM every window;
    the smallest grids have the same block on both sides of a block."""
    kind, Lx, Ly, prm, b, ncol, dt, T, split, init, chunk = case
    F.fskmc_ctx_set_persistent(ctx, chunk)
    F.fskmc_ctx_set_resident(ctx, resident)
    try:
        p = Pair(F, orc, ctx, kind, Lx, Ly, prm, b, ncol, dt, T, split, init=init, seed=0, replica=3)
        p.step_compare_end(3 * chunk + 2)
        p.step_compare_end(chunk)
        F.fskmc_sync(ctx)
    finally:
        F.fskmc_ctx_set_persistent(ctx, 0)
        F.fskmc_ctx_set_resident(ctx, 1)


@pytest.mark.parametrize("L", [2048, 4096], ids=["2048-four-blocks-per-wave", "4096-streaming-fallback"])
def test_resident_many_blocks_per_wave(F, ctx, L):
    """More blocks than resident waves: up to four blocks per wave stay in LDS
    (2048^2, 16384 blocks of 16x16); beyond that (4096^2) the persistent sweep
    falls back to streaming.  Both equal one launch per window."""
    import hashlib
    out = []
    for persist in (0, 12):
        F.fskmc_ctx_set_persistent(ctx, persist)
        try:
            s = F.Sim(ctx, FLIP, L, L, (1.0, 1.0, 1.0, 0.0, 1.0), b=16, n_colours=2, dt=0.1, T=100.0, split=0,
                      seed=0, replica=5)
            s.init(1, 0.5)
            s.advance(12)
            s.advance(12)
            out.append((hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"]))
            s.close()
        finally:
            F.fskmc_ctx_set_persistent(ctx, 0)
    assert out[0] == out[1]


def test_persistent_full_run_config1(F, orc, ctx):
    """The 1024^2 workload's first 40 windows as one persistent launch."""
    F.fskmc_ctx_set_persistent(ctx, 40)
    try:
        p = Pair(F, orc, ctx, FLIP, 1024, 1024, (1.0, 1.0, 1.0, 0.0, 1.0), 16, 2, 0.1, 100.0, "lie",
                 init="bernoulli", seed=0, replica=0)
        p.step_compare_end(40)
    finally:
        F.fskmc_ctx_set_persistent(ctx, 0)


@pytest.mark.parametrize("case", [
    (FLIP, 1024, 1024, (1.0, 1.0, 1.0, 0.0, 1.0), 16, 2, 0.1, 100.0, 0, "bernoulli", 2000, 2000),
    (FLIP, 1024, 1024, (1.0, 1.0, 0.5, 0.0, 1.0), 16, 2, 0.01, 100.0, 1, "bernoulli", 3000, 1000),
    (ZGB, 4096, 4096, (0.5, 1000.0, 10.0), 32, 4, 0.05, 10.0, 1, "empty", 280, 70),
], ids=["config1-full-run", "config1-strang-dt0.01", "config2-280-windows"])
def test_persistent_equals_per_window_at_scale(F, ctx, case):
    """Whole runs at the workloads' full sizes: the persistent sweep and one
    launch per window give identical lattices and event counts."""
    import hashlib
    kind, Lx, Ly, prm, b, ncol, dt, T, split, init, nwin, chunk = case
    out = []
    for persist in (0, chunk):
        F.fskmc_ctx_set_persistent(ctx, persist)
        try:
            s = F.Sim(ctx, kind, Lx, Ly, prm, b=b, n_colours=ncol, dt=dt, T=T, split=split, seed=0, replica=7)
            s.init(1 if init == "bernoulli" else 0, 0.5)
            s.advance(nwin)
            out.append((hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"]))
            s.close()
        finally:
            F.fskmc_ctx_set_persistent(ctx, 0)
    assert out[0] == out[1]


def _golden_full_runs():
    import json
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_runs.json")
    with open(path) as f:
        return json.load(f)


_FULL = _golden_full_runs()


@pytest.mark.parametrize("name", sorted(_FULL))
@pytest.mark.parametrize("persist", [0, 1, 2], ids=["per-window", "persistent-resident", "persistent-streaming"])
def test_full_run_matches_oracle_golden(F, ctx, name, persist):
    """Whole runs at the workloads' full sizes against the oracle's final
    lattice hash and event total (stored by tests/golden/make_full_runs.py,
    which calls only the oracle): one launch per window, and all windows in
    one persistent launch."""
    import hashlib
    g = _FULL[name]
    p = g["params"]
    prm = ((p["k_a"], p["k_d"], p["J"], p["h"], p["beta"]) if g["kind"] == "flip" else
           (p["D"], p["J"], p["beta"]) if g["kind"] == "kawasaki" else (p["y"], p["k_r"], p["D"]))
    F.fskmc_ctx_set_persistent(ctx, g["windows"] if persist else 0)
    F.fskmc_ctx_set_resident(ctx, persist != 2)
    try:
        s = F.Sim(ctx, g["kind"], g.get("Lx", g["L"]), g.get("Ly", g["L"]), prm, b=g["b"], n_colours=g["n_colours"], dt=g["dt"], T=g["T"],
                  split=g["split"], seed=g["seed"], replica=g["replica"])
        s.init(1 if g["init"] == "bernoulli" else 0, 0.5)
        s.advance(g["windows"])
        got = (hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"])
        s.close()
    finally:
        F.fskmc_ctx_set_persistent(ctx, 0)
        F.fskmc_ctx_set_resident(ctx, 1)
    assert got == (g["sha256"], g["events"])


@pytest.mark.parametrize("resident", [1, 0], ids=["resident", "streaming"])
def test_persistent_wait_timeout_reports_edevice(F, ctx, resident):
    """Failure handling forced from the host: with a wait limit of one tick of
    the 100 MHz clock (far below one neighbour hand-off) a persistent sweep
    aborts, every wave leaving its own bounded wait; the next synchronising
    call reports FSKMC_EDEVICE, and afterwards the context and the
    re-initialised simulation give the one-launch-per-window results."""
    import hashlib

    def run(persist):
        F.fskmc_ctx_set_persistent(ctx, persist)
        s.init(1, 0.5)
        s.advance(40)
        return hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"]

    s = F.Sim(ctx, FLIP, 256, 256, (1.0, 1.0, 1.0, 0.0, 1.0), b=16, n_colours=2, dt=0.1, T=100.0, split=0, seed=0,
              replica=1)
    F.fskmc_ctx_set_resident(ctx, resident)
    try:
        F.fskmc_ctx_set_persistent(ctx, 40)
        F.fskmc_ctx_set_wait_limit(ctx, 1e-8)
        s.init(1, 0.5)
        s.advance(40)
        with pytest.raises(F.FskmcError) as err:
            F.fskmc_sync(ctx)
        assert err.value.code == F.FSKMC_EDEVICE
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        assert run(40) == run(0)
    finally:
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        F.fskmc_ctx_set_persistent(ctx, 0)
        F.fskmc_ctx_set_resident(ctx, 1)
        s.close()


@pytest.mark.parametrize("L,chunk", [(512, 25), (2048, 10)], ids=["512-pairs", "2048-capacity-bound"])
def test_rebalanced_resident(F, ctx, L, chunk):
    """Workload rebalancing (Sec. 6) on a half-filled lattice (the empty half
    adsorbs, the full half is nearly idle): every resident launch takes its
    block ranges from the oracle's mass-transport map of the block costs of
    the previous launch (jumps plus 3 per window of the block's colour; an
    even split the first time), and the run is bit-for-bit the
    one-launch-per-window run."""
    import hashlib
    from oracle import balance
    N = L * L
    lat0 = np.zeros(N, np.uint8)
    lat0[N // 2:] = 1
    prm = (1.0, 1.0, 1.0, 0.0, 1.0)
    cap = 8  # blocks a wave holds for 16x16 blocks

    def sim():
        s = F.Sim(ctx, FLIP, L, L, prm, b=16, n_colours=2, dt=0.1, T=100.0, split=0, seed=0, replica=9)
        s.set_lattice(lat0)
        return s

    ref = sim()
    ref.advance(4 * chunk)
    want = (hashlib.sha256(ref.lattice().tobytes()).hexdigest(), ref.observe()["events"])
    ref.close()
    s = sim()
    F.fskmc_ctx_set_persistent(ctx, chunk)
    F.fskmc_ctx_set_rebalance(ctx, 1)
    NBX = L // 16
    colours = [((m % NBX) + (m // NBX)) % 2 for m in range(NBX * NBX)]  # Lie: window w has colour w % 2
    active = [(chunk + 1) // 2, chunk // 2]  # windows of each colour in a launch starting at an even window
    try:
        prev = s.workload()
        assert not prev.any()
        cost = [1] * s.nb
        for k in range(4):
            s.advance(chunk)
            part = s.last_partition()
            now = s.workload()
            waves = len(part) - 1
            use = min(waves, max((s.nb + 1) // 2, -(-s.nb // cap)))
            expect = balance.cdf_partition(cost, use, cap) + [s.nb] * (waves - use)
            assert part.tolist() == expect, k
            W, prev = now - prev, now
            act = active if (k * chunk) % 2 == 0 else active[::-1]
            cost = balance.block_costs(W.tolist(), colours, act, 3)
            if k == 0:
                first = W.copy()
        got = (hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"])
    finally:
        F.fskmc_ctx_set_rebalance(ctx, 0)
        F.fskmc_ctx_set_persistent(ctx, 0)
        s.close()
    assert got == want
    half = len(first) // 2
    assert first[:half].sum() > 10 * first[half:].sum()  # the first histogram is strongly unbalanced
