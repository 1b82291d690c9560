"""ctypes loader for liblmmse.so: the prototypes of include/lmmse.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmmse.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
P_int = ctypes.POINTER(ctypes.c_int)
P_double = ctypes.POINTER(ctypes.c_double)
P_size_t = ctypes.POINTER(ctypes.c_size_t)

# lmmse_status
OK, INVALID_ARG, UNSUPPORTED, WORKSPACE, HIP, NOT_PD, NOT_READY, NO_DEVICE, RANGE = range(9)
# lmmse_rsource
R_UNIFORM, R_EXPONENTIAL, R_SAMPLE, R_USER, R_USER_R = range(5)
# lmmse_precision
FP32, BF16X3, FP16X3 = range(3)
# size of the static workspace of lmmse_estimate_noalloc (LMMSE_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("M", c_int), ("K", c_int), ("N", c_int), ("N_fft", c_int),
        ("B", c_int), ("Wn", c_int), ("rsource", c_int), ("precision", c_int),
        ("max_slots", c_int), ("taps", c_int),
        ("tau_rms", c_double), ("L", c_double), ("sigma2", c_double),
    ]


P_desc = ctypes.POINTER(PlanDesc)

# lmmse_comb_kind
COMB_3W, COMB_12W, COMB_LS_HOLD, COMB_LS_LINEAR, COMB_LS_LINEAR3, COMB_LS_QUADRATIC, COMB_LS_SPLINE = range(7)


class CombDesc(ctypes.Structure):
    _fields_ = [
        ("M", c_int), ("K", c_int), ("comb", c_int), ("N", c_int), ("N_fft", c_int),
        ("kind", c_int), ("rsource", c_int), ("taps", c_int),
        ("tau_rms", c_double), ("L", c_double), ("sigma2", c_double), ("max_slots", c_int),
    ]


P_cdesc = ctypes.POINTER(CombDesc)

# name -> (restype, argtypes); mirrors include/lmmse.h
PROTOTYPES = {
    "lmmse_status_string": (ctypes.c_char_p, [c_int]),
    "lmmse_version": (c_int, []),
    "lmmse_plan_validate": (c_int, [P_desc]),
    "lmmse_block_plan": (c_int, [c_int, c_int, c_int, P_int, P_int, P_int, P_int]),
    "lmmse_workspace_size": (c_int, [P_desc, c_int, P_size_t]),
    "lmmse_plan_create": (c_int, [P_desc, ctypes.POINTER(c_void_p)]),
    "lmmse_plan_destroy": (c_int, [c_void_p]),
    "lmmse_plan_get_desc": (c_int, [c_void_p, P_desc]),
    "lmmse_set_design": (c_int, [c_void_p, c_double, c_double, c_void_p]),
    "lmmse_set_filters": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lmmse_get_filters": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lmmse_despread": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lmmse_apply": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "lmmse_covariance": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "lmmse_sample_filters_workspace_size": (c_int, [P_desc, c_int, P_size_t]),
    "lmmse_sample_filters": (c_int, [c_void_p, c_int, c_void_p, c_double, c_void_p, c_void_p,
                                     c_size_t, c_void_p]),
    "lmmse_set_correlation": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lmmse_set_input_scale": (c_int, [c_void_p, c_double]),
    "lmmse_estimate_ls": (c_int, [c_void_p, c_int, c_void_p, c_double, c_void_p, c_void_p,
                                  c_size_t, c_void_p]),
    "lmmse_estimate": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_double, c_void_p,
                               c_void_p, c_size_t, c_void_p]),
    "lmmse_estimate_noalloc": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_double, c_void_p,
                                       c_void_p]),
    "lmmse_backward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, P_double,
                               P_double, c_void_p, c_size_t, c_void_p]),
    "lmmse_backward_dev": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    "lmmse_design_state_size": (c_int, [c_void_p, c_int, P_size_t]),
    "lmmse_estimate_ls_keep": (c_int, [c_void_p, c_int, c_void_p, c_double, c_void_p, c_void_p,
                                       c_size_t, c_void_p, c_size_t, c_void_p]),
    "lmmse_backward_kept": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "lmmse_sync_status": (c_int, [c_void_p, c_void_p, P_int]),
    "lmmse_comb_validate": (c_int, [P_cdesc]),
    "lmmse_comb_create": (c_int, [P_cdesc, ctypes.POINTER(c_void_p)]),
    "lmmse_comb_destroy": (c_int, [c_void_p]),
    "lmmse_comb_get_filters": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lmmse_comb_estimate": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lmmse_mmse_detect": (c_int, [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_double,
                                  c_void_p, c_void_p]),
}

_LIB = None


class LmmseError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


def load() -> ctypes.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1802_05427_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def status_string(status: int) -> str:
    return load().lmmse_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != OK:
        raise LmmseError(status, where)
