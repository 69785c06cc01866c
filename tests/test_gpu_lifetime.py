"""Object lifetimes and failure bookkeeping of libfskmc on the GPU, through
the C ABI.

* Destroying a context destroys the simulations still created on it; the
  Python objects of those simulations are closed with it, and closing them
  afterwards is a no-op (no use of freed memory).
* The abort flag of the persistent sweeps is sticky: an aborted launch
  followed, before any synchronisation, by a launch that finishes cleanly is
  still reported by the next synchronising call (FSKMC_EDEVICE), every
  simulation those launches advanced is marked invalid (FSKMC_ESTATE) until
  it is re-initialised, and afterwards the results are the
  one-launch-per-window results again.

The aborts are forced from the host with a wait limit of one tick of the
100 MHz clock: every wave leaves through its own bounded wait.
"""
import ctypes
import hashlib

import pytest

pytestmark = pytest.mark.gpu

PRM = (1.0, 1.0, 1.0, 0.0, 1.0)


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


def _digest(s):
    return hashlib.sha256(s.lattice().tobytes()).hexdigest(), s.observe()["events"]


def test_ctx_destroy_releases_its_sims(F):
    ctx = F.fskmc_ctx_create(0)
    sims = [F.Sim(ctx, "flip", 128, 128, PRM, b=16, n_colours=2, dt=0.1, T=10.0, split=0, seed=0, replica=r)
            for r in range(3)]
    for s in sims:
        s.init(1, 0.5)
        s.advance(10)
    sims[0].close()
    F.fskmc_ctx_destroy(ctx)
    assert all(s.handle is None for s in sims)
    for s in sims:
        s.close()  # no-op: released with the context

    # the same through the raw C ABI: a sim left behind is freed by the
    # context, and a fresh context afterwards gives the same bits
    L = F.lib
    raw = ctypes.c_void_p()
    assert L.fskmc_ctx_create(0, None, ctypes.byref(raw)) == F.FSKMC_OK
    lat = F.fskmc_lattice(2, 128, 128)
    p = F.fskmc_flip_params(*PRM)
    dec = F.fskmc_decomp(16, 16, 2, None)
    sch = F.fskmc_schedule(0.1, 10.0, 0)
    sim = ctypes.c_void_p()
    assert L.fskmc_sim_create(raw, ctypes.byref(lat), F.FSKMC_MODEL_FLIP, ctypes.cast(ctypes.byref(p), ctypes.c_void_p),
                              ctypes.byref(dec), ctypes.byref(sch), F.fskmc_key(0, 1), ctypes.byref(sim)) == F.FSKMC_OK
    assert L.fskmc_sim_init(sim, 1, ctypes.c_double(0.5)) == F.FSKMC_OK
    assert L.fskmc_sim_advance(sim, 10) == F.FSKMC_OK
    assert L.fskmc_ctx_destroy(raw) == F.FSKMC_OK

    ctx = F.fskmc_ctx_create(0)
    try:
        a = F.Sim(ctx, "flip", 128, 128, PRM, b=16, n_colours=2, dt=0.1, T=10.0, split=0, seed=0, replica=1)
        a.init(1, 0.5)
        a.advance(10)
        b = F.Sim(ctx, "flip", 128, 128, PRM, b=16, n_colours=2, dt=0.1, T=10.0, split=0, seed=0, replica=1)
        b.init(1, 0.5)
        b.advance(10)
        assert _digest(a) == _digest(b)
    finally:
        F.fskmc_ctx_destroy(ctx)


@pytest.mark.parametrize("resident", [1, 0], ids=["resident", "streaming"])
def test_abort_is_sticky_across_launches(F, resident):
    ctx = F.fskmc_ctx_create(0)
    try:
        F.fskmc_ctx_set_resident(ctx, resident)
        s = F.Sim(ctx, "flip", 512, 512, PRM, b=16, n_colours=2, dt=0.1, T=100.0, split=0, seed=0, replica=4)
        other = F.Sim(ctx, "flip", 128, 128, PRM, b=16, n_colours=2, dt=0.1, T=100.0, split=0, seed=0, replica=5)
        F.fskmc_ctx_set_persistent(ctx, 20)
        s.init(1, 0.5)
        other.init(1, 0.5)
        F.fskmc_sync(ctx)
        F.fskmc_ctx_set_wait_limit(ctx, 1e-8)
        s.advance(20)               # aborts
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        s.advance(20)               # enqueued before any synchronisation
        other.advance(20)           # a second sim in the same interval
        with pytest.raises(F.FskmcError) as err:
            F.fskmc_sync(ctx)
        assert err.value.code == F.FSKMC_EDEVICE
        F.fskmc_sync(ctx)  # reported once, then cleared
        for sim in (s, other):
            for call in (lambda: sim.advance(1), sim.observe, sim.lattice, sim.workload, sim.block_events):
                with pytest.raises(F.FskmcError) as err:
                    call()
                assert err.value.code == F.FSKMC_ESTATE
        with pytest.raises(F.FskmcError) as err:
            F.fskmc_batch_advance(ctx, [s.handle], 1)
        assert err.value.code == F.FSKMC_ESTATE

        # re-initialised, the sim is valid again and gives the per-window bits
        s.init(1, 0.5)
        s.advance(40)
        got = _digest(s)
        F.fskmc_ctx_set_persistent(ctx, 0)
        s.init(1, 0.5)
        s.advance(40)
        assert got == _digest(s)
        s.close()
        other.close()
    finally:
        F.fskmc_ctx_destroy(ctx)


def test_batched_abort_is_sticky(F):
    ctx = F.fskmc_ctx_create(0)
    try:
        F.fskmc_ctx_set_batch_persistent(ctx, 10)
        sims = [F.Sim(ctx, "flip", L, L, PRM, b=16, n_colours=2, dt=0.1, T=10.0, split=0, seed=0, replica=r)
                for r, L in enumerate((1024, 128))]
        for x in sims:
            x.init(1, 0.5)
        F.fskmc_sync(ctx)
        h = [x.handle for x in sims]
        F.fskmc_ctx_set_wait_limit(ctx, 1e-8)
        F.fskmc_batch_advance(ctx, h, 10)  # aborts
        F.fskmc_ctx_set_wait_limit(ctx, 2.0)
        F.fskmc_batch_advance(ctx, h, 10)  # clean, before any synchronisation
        with pytest.raises(F.FskmcError) as err:
            F.fskmc_sync(ctx)
        assert err.value.code == F.FSKMC_EDEVICE
        with pytest.raises(F.FskmcError) as err:
            F.fskmc_batch_advance(ctx, h, 1)
        assert err.value.code == F.FSKMC_ESTATE
        for x in sims:
            x.init(1, 0.5)
        F.fskmc_batch_advance(ctx, h, 20)
        got = [_digest(x) for x in sims]
        F.fskmc_ctx_set_batch_persistent(ctx, 0)
        for x in sims:
            x.init(1, 0.5)
            x.advance(20)
        assert got == [_digest(x) for x in sims]
    finally:
        F.fskmc_ctx_destroy(ctx)
