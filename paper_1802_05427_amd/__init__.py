"""Partitioned LMMSE channel estimation for the massive-MIMO OFDM uplink on
MI355X (gfx950): a C-ABI HIP library (liblmmse.so, include/lmmse.h) and a
thin torch binding.  Importing this package does not touch the GPU; creating
a Plan loads the library and fails loudly if it has not been built.
"""
from ._lib import LmmseError, load  # noqa: F401
from .api import CombPlan, Plan, block_plan, comb_validate, make_desc, workspace_size  # noqa: F401

__all__ = ["Plan", "CombPlan", "block_plan", "comb_validate", "make_desc", "workspace_size",
           "LmmseError", "load"]
