"""Partitioned LMMSE channel estimation for the massive-MIMO OFDM uplink on
MI355X (gfx950): a C-ABI HIP library (liblmmse.so, include/lmmse.h) and a
thin torch binding.  Importing this package does not touch the GPU; creating
a Plan loads the library and fails loudly if it has not been built.
"""
from ._lib import LmmseError, load  # noqa: F401
from .api import (  # noqa: F401
    CombPlan, Plan, block_plan, comb_validate, make_desc, mmse_detect, workspace_size)

__all__ = ["Plan", "CombPlan", "block_plan", "comb_validate", "make_desc", "mmse_detect", "workspace_size",
           "LmmseError", "load"]
