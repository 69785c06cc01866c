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
                   "fskmc_ctx_set_batch_persistent", "fskmc_ctx_set_graphs", "fskmc_ctx_set_rebalance"):
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

