"""Host paths of libfskmc that need no GPU: argument checks behind the C ABI
return their error codes with a message, the footprint of a simulation is
computed on the host, and creating a context without a device fails cleanly
with FSKMC_EDEVICE (this container has no GPU; on a GPU machine that case is
skipped)."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def F():
    from paper_1105_4673_amd import fskmc
    return fskmc


def test_null_arguments_are_rejected(F):
    L = F.lib
    assert L.fskmc_sync(None) == F.FSKMC_EINVAL and b"NULL" in L.fskmc_last_error()
    key = F.fskmc_key(0, 0)
    assert L.fskmc_sim_create(None, None, 1, None, None, None, key, None) == F.FSKMC_EINVAL
    assert L.fskmc_sim_create_nested(None, None, 1, None, None, None, key, None) == F.FSKMC_EINVAL
    assert L.fskmc_sim_advance(None, 1) == F.FSKMC_EINVAL
    assert L.fskmc_sim_observe(None, None) == F.FSKMC_EINVAL
    assert L.fskmc_batch_advance(None, None, 1, 1) == F.FSKMC_EINVAL
    for setter in ("fskmc_ctx_set_persistent", "fskmc_ctx_set_resident", "fskmc_ctx_set_nested",
                   "fskmc_ctx_set_batch_persistent", "fskmc_ctx_set_graphs", "fskmc_ctx_set_rebalance",
                   "fskmc_ctx_set_batch_streams"):
        assert getattr(L, setter)(None, 1) == F.FSKMC_EINVAL, setter
    assert L.fskmc_sim_destroy(None) == F.FSKMC_OK and L.fskmc_ctx_destroy(None) == F.FSKMC_OK


def test_footprint_on_the_host(F):
    L = F.lib
    lat = F.fskmc_lattice(2, 64, 64)
    dec = F.fskmc_decomp(8, 8, 2, None)
    small = L.fskmc_sim_footprint(ctypes.byref(lat), 1, ctypes.byref(dec), ctypes.byref(F.fskmc_schedule(0.1, 1.0, 0)))
    long_ = L.fskmc_sim_footprint(ctypes.byref(lat), 1, ctypes.byref(dec), ctypes.byref(F.fskmc_schedule(0.1, 10.0, 0)))
    assert 4096 < small < long_  # the lattice, plus per-window tables that grow with T
    bad = F.fskmc_schedule(0.0, 1.0, 0)
    assert L.fskmc_sim_footprint(ctypes.byref(lat), 1, ctypes.byref(dec), ctypes.byref(bad)) == 0


def test_context_without_a_device(F):
    try:
        import torch
        if torch.cuda.device_count() > 0:
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(F.FskmcError) as ei:
        F.fskmc_ctx_create(0)
    assert ei.value.code == F.FSKMC_EDEVICE



def test_noalloc_arguments_are_checked_before_any_hip_call(F):
    """The allocation-free advance rejects every bad argument on the host
    (these calls never reach the device, so they run without a GPU)."""
    flip = (1.0, 1.0, 1.0, 0.0, 1.0)
    fake = 0x1000  # never dereferenced: every case below fails its checks first

    def call(Lx=64, Ly=64, model=F.FSKMC_MODEL_FLIP, params=flip, b=16, K=2, dt=0.1, T=1.0, split=0, w0=0, n=4,
             lat=fake):
        try:
            F.fskmc_advance_noalloc(0, None, 1 if Ly == 1 else 2, Lx, Ly, model, params, b, b if Ly > 1 else 1, K,
                                    dt, T, split, 0, 0, lat, w0, n)
        except F.FskmcError as e:
            return e.code
        return F.FSKMC_OK

    assert call(lat=0) == F.FSKMC_EINVAL                      # no lattice
    assert call(Lx=8192, Ly=8192, b=16) == F.FSKMC_EINVAL     # 262144 blocks > the static scratch
    assert call(b=12) == F.FSKMC_EINVAL                       # no kernel for 12x12 blocks
    assert call(K=3) == F.FSKMC_EINVAL                        # built-in maps only
    assert call(Lx=48, Ly=64) == F.FSKMC_EDECOMP              # 3 block columns: same colour across the wrap
    assert call(model=F.FSKMC_MODEL_ZGB, params=(0.5, 1000.0, 10.0), b=32, K=2) == F.FSKMC_EDECOMP  # corners
    assert call(T=1.05, dt=0.1) == F.FSKMC_EINVAL             # T / dt not an integer
    assert call(w0=18, n=4) == F.FSKMC_ESTATE                 # 20 windows in the schedule
    assert call(params=(1.0, -1.0, 1.0, 0.0, 1.0)) == F.FSKMC_EINVAL
    L = F.lib
    with_map = F.fskmc_decomp(16, 16, 2, (ctypes.c_int * 16)(*([0, 1, 0, 1, 1, 0, 1, 0] * 2)))
    lat = F.fskmc_lattice(2, 64, 64)
    p = F.fskmc_flip_params(*flip)
    rc = L.fskmc_advance_noalloc(0, None, ctypes.byref(lat), F.FSKMC_MODEL_FLIP,
                                 ctypes.cast(ctypes.byref(p), ctypes.c_void_p), ctypes.byref(with_map),
                                 ctypes.byref(F.fskmc_schedule(0.1, 1.0, 0)), F.fskmc_key(0, 0),
                                 ctypes.c_void_p(fake), 0, 1, None, None)
    assert rc == F.FSKMC_EINVAL and b"built-in" in L.fskmc_last_error()
