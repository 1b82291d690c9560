"""FP64 CPU oracle of the partitioned LMMSE channel estimator.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or runs
anything in this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP library.

Everything here is plain NumPy/SciPy in complex128, written step by step from
the paper (Sec. IV-A: LS eq. 8-9, LMMSE eq. 12-15, fixed design eq. 16 /
r_d and eq. 17; Sec. IV-B: partitioning of the correlation matrix into small
overlapping or non-overlapping blocks, Tables I-II; the comb-pilot 3W / 12W
estimators of Sec. IV-B in comb.py; MMSE detection, eq. 20-22, in detect.py)
plus the readings of the points the paper
leaves open, which are listed in each function.
"""
from .lmmse import (  # noqa: F401
    apply_filters,
    block_filters,
    comb_group_table,
    cover_code,
    despread,
    discrepancy_db,
    estimate,
    expected_mse,
    full_lmmse_filter,
    nmse,
    nmse_db,
    r_exponential,
    r_exponential_cont,
    r_uniform,
    sample_covariance,
    toeplitz_from_r,
    window_starts,
)
from .comb import (  # noqa: F401
    comb_estimate,
    comb_filters,
    comb_groups,
    comb_ls,
    comb_ls_hold,
    comb_ls_linear,
    comb_ls_quadratic,
    comb_ls_spline,
    natural_spline_second_derivatives,
    zero_order_hold,
)
from .detect import mmse_detect, qpsk_decide  # noqa: F401
from .fit_optimum import design_mse, fit_optimum, mixture_r  # noqa: F401
from .grad import (  # noqa: F401
    dr_exponential_dtau,
    grad_fixed_design,
    grad_sample_cov,
    mse_loss_and_grad,
)
