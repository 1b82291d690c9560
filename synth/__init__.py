"""Seeded synthetic uplink pilot slots (inputs only; no estimator arithmetic).

This package draws channels, pilots and noise with the statistics of the
paper's system model (Sec. II, eq. 1-5; exponential power-delay profile of
Sec. IV-A) and the code-division pilot layout used by this project.  Both the
FP64 oracle tests and the GPU path consume what it produces; it computes
nothing that the estimator computes.
"""
from .slots import (  # noqa: F401
    CONFIGS,
    PILOT_SEED,
    SlotBatch,
    exponential_pdp,
    CombBatch,
    make_comb_batch,
    make_config_batch,
    make_data_symbols,
    make_pilots,
    make_slot_batch,
    slot_seed,
)
