"""Batched advances (needs a GPU): one packed launch per window (the
full-launch and the 16-sites-per-lane small-launch kernels), the persistent
batched sweep (K windows of every sim per launch, work items from a device
counter) and HIP-graph replay of the batch's launch sequence give every sim
the oracle's bits (final lattice and event total of the blockwise scheme,
Sec. 2.2 eq. exact) and the bits it gets alone."""
import hashlib
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FLIP, ZGB, KAW = "flip", "zgb", "kawasaki"

SPECS = [
    dict(kind=FLIP, Lx=128, Ly=128, params=(1.0, 1.0, 1.5, -0.5, 1.0), b=16, n_colours=2, dt=0.1, T=2.0, split=0,
         seed=0, replica=1),
    dict(kind=FLIP, Lx=256, Ly=256, params=(1.0, 1.0, 0.3, 0.8, 1.0), b=16, n_colours=2, dt=0.2, T=2.0, split=1,
         seed=0, replica=2),
    dict(kind=FLIP, Lx=64, Ly=64, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=8, n_colours=2, dt=0.1, T=3.0, split=2,
         seed=0, replica=3),
    dict(kind=ZGB, Lx=128, Ly=128, params=(0.5, 1000.0, 10.0), b=32, n_colours=4, dt=0.05, T=1.0, split=1, seed=0,
         replica=4),
    dict(kind=FLIP, Lx=512, Ly=1, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=64, n_colours=2, dt=1.0, T=5.0, split=0,
         seed=0, replica=5),
    dict(kind=KAW, Lx=128, Ly=128, params=(4.0, 1.0, 1.0), b=16, n_colours=4, dt=0.25, T=3.0, split=1, seed=0,
         replica=6),
    dict(kind=FLIP, Lx=1024, Ly=1024, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=16, n_colours=2, dt=0.1, T=1.0, split=0,
         seed=0, replica=7),
]


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


@pytest.fixture()
def ctx(F):
    c = F.fskmc_ctx_create(0)
    yield c
    F.fskmc_ctx_destroy(c)


def _make(F, ctx, specs):
    sims = []
    for sp in specs:
        s = F.Sim(ctx, **sp)
        s.init(1, 0.5)
        sims.append(s)
    return sims


def _digest(s):
    return hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"]


sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _oracle_jobs import oracle_result  # noqa: E402


def _oracle(orc, specs):
    """The oracle's (sha256, events) of each whole run; _make starts every
    sim from the Bernoulli(1/2) state."""
    return [oracle_result(orc, dict(sp, init="bernoulli")) for sp in specs]


def _alone(F, ctx, specs):
    out = []
    for s in _make(F, ctx, specs):
        s.run_to_end()
        out.append(_digest(s))
        s.close()
    return out


@pytest.mark.parametrize("K", [0, 1, 3, 50])
@pytest.mark.parametrize("graphs", [1, 0], ids=["graph", "eager"])
def test_batch_persistent_equals_alone(F, orc, ctx, K, graphs):
    """K = 0: one packed launch per window (k_sweep_batched; the reaction job
    of 32x32 blocks takes the small-launch kernel for 16 sites per lane);
    K > 0: k_sweep_batched_persistent, K windows per launch."""
    want = _alone(F, ctx, SPECS)
    assert want == _oracle(orc, SPECS)
    F.fskmc_ctx_set_batch_persistent(ctx, K)
    F.fskmc_ctx_set_graphs(ctx, graphs)
    sims = _make(F, ctx, SPECS)
    handles = [s.handle for s in sims]
    while any(s.windows()[1] < s.windows()[0] for s in sims):
        F.fskmc_batch_advance(ctx, handles, 7)
    F.fskmc_sync(ctx)
    got = [_digest(s) for s in sims]
    for s in sims:
        s.close()
    assert got == want


@pytest.mark.parametrize("streams", [1, 2, 4])
@pytest.mark.parametrize("graphs", [1, 0], ids=["graph", "eager"])
def test_batch_streams_equal_alone(F, orc, ctx, streams, graphs):
    """The five kernel-variant groups of SPECS (spin flip on 16x16, 8x8 and
    1D blocks, the reaction model on 32x32, spin exchange on 16x16) with 1, 2
    or 4 streams: launched directly the groups spread over that many streams,
    replayed from a graph they stay on the context's stream; either way every
    sim gets the oracle's bits."""
    F.fskmc_ctx_set_batch_persistent(ctx, 0)
    F.fskmc_ctx_set_batch_streams(ctx, streams)
    F.fskmc_ctx_set_graphs(ctx, graphs)
    sims = _make(F, ctx, SPECS)
    while any(s.windows()[1] < s.windows()[0] for s in sims):
        F.fskmc_batch_advance(ctx, [s.handle for s in sims], 6)
    F.fskmc_sync(ctx)
    got = [_digest(s) for s in sims]
    for s in sims:
        s.close()
    assert got == _oracle(orc, SPECS)


def test_batch_full_and_small_launch_kernels(F, orc, ctx):
    """16 sites per lane in both launch kernels at once: the spin-flip group
    holds 2112 blocks per window (the full-launch kernel), the reaction group
    16 (the small-launch kernel); every sim gets the oracle's bits (the
    2112x2048 run's stored value, the reaction job's computed here) and the
    bits it gets alone."""
    specs = [dict(kind=FLIP, Lx=2112, Ly=2048, params=(1.0, 1.0, 0.8, -0.2, 1.0), b=32, n_colours=2, dt=0.2, T=1.0,
                  split=0, seed=0, replica=21),
             dict(kind=ZGB, Lx=256, Ly=256, params=(0.5, 1000.0, 10.0), b=32, n_colours=4, dt=0.05, T=0.5, split=1,
                  seed=0, replica=22)]
    want = _alone(F, ctx, specs)
    assert want == _oracle(orc, specs)
    F.fskmc_ctx_set_batch_persistent(ctx, 0)
    sims = _make(F, ctx, specs)
    while any(s.windows()[1] < s.windows()[0] for s in sims):
        F.fskmc_batch_advance(ctx, [s.handle for s in sims], 4)
    F.fskmc_sync(ctx)
    got = [_digest(s) for s in sims]
    for s in sims:
        s.close()
    assert got == want


@pytest.mark.parametrize("K", [0, 4])
def test_graph_replays_match_eager(F, orc, ctx, K):
    """Two copies of one batch, one replaying a captured graph and one
    launching eagerly, compared after every call (each call uploads a new job
    table and synchronises between the replays)."""
    F.fskmc_ctx_set_batch_persistent(ctx, K)
    a = _make(F, ctx, SPECS[:4])
    b = _make(F, ctx, SPECS[:4])
    calls = 0
    while any(s.windows()[1] < s.windows()[0] for s in a):
        F.fskmc_ctx_set_graphs(ctx, 1)
        F.fskmc_batch_advance(ctx, [s.handle for s in a], 5)
        F.fskmc_sync(ctx)
        F.fskmc_ctx_set_graphs(ctx, 0)
        F.fskmc_batch_advance(ctx, [s.handle for s in b], 5)
        F.fskmc_sync(ctx)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.lattice(), y.lattice())
        calls += 1
    assert calls >= 3
    assert [_digest(x) for x in a] == _oracle(orc, SPECS[:4])
    for s in a + b:
        s.close()


def test_batch_persistent_wait_timeout_reports_edevice(F, orc, ctx):
    """A wait limit far below one window forces the bounded neighbour wait to
    give up: the launch aborts, every wave leaves, the next synchronising call
    reports FSKMC_EDEVICE, and the context works again afterwards."""
    F.fskmc_ctx_set_batch_persistent(ctx, 20)
    sims = _make(F, ctx, SPECS[-1:])
    F.fskmc_ctx_set_wait_limit(ctx, 1e-8)
    try:
        F.fskmc_batch_advance(ctx, [s.handle for s in sims], 10)
        with pytest.raises(F.FskmcError) as ei:
            F.fskmc_sync(ctx)
        assert ei.value.code == F.FSKMC_EDEVICE
    finally:
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
    for s in sims:
        s.close()
    want = _alone(F, ctx, SPECS[:1])
    sims = _make(F, ctx, SPECS[:1])
    while sims[0].windows()[1] < sims[0].windows()[0]:
        F.fskmc_batch_advance(ctx, [sims[0].handle], 9)
    F.fskmc_sync(ctx)
    assert [_digest(sims[0])] == want == _oracle(orc, SPECS[:1])
    sims[0].close()


def test_batch_knobs_invalid(F, ctx):
    with pytest.raises(F.FskmcError) as ei:
        F.fskmc_ctx_set_batch_persistent(ctx, -1)
    assert ei.value.code == F.FSKMC_EINVAL
    for bad in (0, 5):
        with pytest.raises(F.FskmcError) as ei:
            F.fskmc_ctx_set_batch_streams(ctx, bad)
        assert ei.value.code == F.FSKMC_EINVAL


def test_autotune_windows_per_launch_picks_a_candidate(F, ctx):
    from paper_1105_4673_amd import autotune
    best, timings = autotune.tune_windows_per_launch(ctx, lambda: _make(F, ctx, SPECS[:3]), candidates=(0, 5),
                                                      windows=10)
    assert best in (0, 5) and set(timings) == {0, 5} and all(t > 0 for t in timings.values())
    F.fskmc_ctx_set_batch_persistent(ctx, 0)


def test_autotune_block_edges_returns_a_tiling_assignment(F, ctx):
    from paper_1105_4673_amd import autotune
    jobs = [dict(sp, replica=10 + i) for i, sp in enumerate(SPECS[:2] * 2)]

    def make(j, b):
        s = F.Sim(ctx, **dict(j, b=b))
        s.init(1, 0.5)
        return s

    assign, scores = autotune.tune_block_edges(ctx, jobs, make, candidates=(8, 16), class_sample=2, sample=4,
                                               windows=4)
    assert set(assign) == {(128, 128), (256, 256)} and set(assign.values()) <= {8, 16}
    assert scores["chosen"] in scores["assignments"] and {"per-class", "all-b8", "all-b16"} <= set(scores["assignments"])
