"""libfskmc: fractional-step parallel lattice kinetic Monte Carlo on MI355X.

The compute path is the HIP library ``libfskmc.so`` (C ABI in
``include/fskmc.h``); ``fskmc`` is its ctypes binding.  Importing
``paper_1105_4673_amd.fskmc`` fails if the library has not been built.
"""
__all__ = ["fskmc"]
