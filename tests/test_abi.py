"""The C-ABI library loads and exports every entry point include/fskmc.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fskmc.h")
LIB = os.path.join(ROOT, "paper_1105_4673_amd", "libfskmc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fskmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fskmc_ctx_create", "fskmc_sim_create", "fskmc_sim_advance", "fskmc_sim_observe",
                     "fskmc_batch_advance", "fskmc_sim_get_state", "fskmc_sim_set_state"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libfskmc.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1105_4673_amd import fskmc
    assert sorted(fskmc.SYMBOLS) == declared_functions()
    for name in declared_functions():
        if name != "fskmc_last_error":
            assert callable(getattr(fskmc, name)), name


def test_footprint_is_host_only():
    from paper_1105_4673_amd import fskmc
    n = fskmc.fskmc_sim_footprint(2, 1024, 1024, fskmc.FSKMC_MODEL_FLIP, 16, 16, 2, 0.1, 100.0, fskmc.FSKMC_LIE)
    assert n >= 1024 * 1024
    assert fskmc.fskmc_sim_footprint(2, 1024, 1024, fskmc.FSKMC_MODEL_FLIP, 0, 16, 2, 0.1, 1.0, 0) == 0


def test_last_error_is_a_string():
    from paper_1105_4673_amd import fskmc
    assert isinstance(fskmc.lib.fskmc_last_error(), bytes)
