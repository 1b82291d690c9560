"""Thin Python binding of the C ABI over torch tensors.

Argument marshalling only: shapes, dtypes and devices are checked, device
pointers and the current HIP stream are passed to liblmmse.so, and every step
of the estimator runs in the library's kernels.  Torch supplies device memory
(including the workspace) and the stream.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from ._lib import CombDesc, PlanDesc, check

_RSOURCE = {"uniform": _lib.R_UNIFORM, "exp": _lib.R_EXPONENTIAL,
            "sample": _lib.R_SAMPLE, "user": _lib.R_USER, "user_r": _lib.R_USER_R}
_PREC = {"fp32": _lib.FP32, "bf16x3": _lib.BF16X3, "fp16x3": _lib.FP16X3}


def make_desc(M, K, N, N_fft, B, Wn, rsource="exp", precision="fp32", max_slots=1,
              taps=1, tau_rms=1.0, L=1.0, sigma2=0.1) -> PlanDesc:
    return PlanDesc(M=int(M), K=int(K), N=int(N), N_fft=int(N_fft), B=int(B), Wn=int(Wn),
                    rsource=_RSOURCE[rsource] if isinstance(rsource, str) else int(rsource),
                    precision=_PREC[precision] if isinstance(precision, str) else int(precision),
                    max_slots=int(max_slots), taps=int(taps), tau_rms=float(tau_rms),
                    L=float(L), sigma2=float(sigma2))


def block_plan(N: int, B: int, Wn: int):
    """(starts, offsets, classes, n_classes) of the block plan (host only)."""
    lib = _lib.load()
    nb = N // B if B > 0 else 0
    s = (ctypes.c_int * max(nb, 1))()
    o = (ctypes.c_int * max(nb, 1))()
    c = (ctypes.c_int * max(nb, 1))()
    n = ctypes.c_int(0)
    check(lib.lmmse_block_plan(N, B, Wn, s, o, c, ctypes.byref(n)), "lmmse_block_plan")
    return list(s[:nb]), list(o[:nb]), list(c[:nb]), n.value


def workspace_size(desc: PlanDesc, slots: int) -> int:
    lib = _lib.load()
    b = ctypes.c_size_t(0)
    check(lib.lmmse_workspace_size(ctypes.byref(desc), int(slots), ctypes.byref(b)),
          "lmmse_workspace_size")
    return b.value


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """An estimator plan on the current GPU (see include/lmmse.h)."""

    def __init__(self, **kw):
        self._lib = _lib.load()
        self.desc = make_desc(**kw)
        h = ctypes.c_void_p()
        check(self._lib.lmmse_plan_create(ctypes.byref(self.desc), ctypes.byref(h)),
              "lmmse_plan_create")
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.starts, self.offsets, self.classes, self.n_classes = block_plan(
            self.desc.N, self.desc.B, self.desc.Wn)
        if self.desc.rsource == _lib.R_USER_R:   # one filter per block
            self.classes, self.n_classes = list(range(self.nb)), self.nb
        self._ws = None

    # ---- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.lmmse_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- helpers
    @property
    def nb(self) -> int:
        return self.desc.N // self.desc.B

    def _check_cols(self, t: torch.Tensor, name: str) -> int:
        d = self.desc
        if t.dtype != torch.complex64 or t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor")
        if t.dim() != 4 or tuple(t.shape[1:]) != (d.M, d.K, d.N):
            raise ValueError(f"{name} must be [S, {d.M}, {d.K}, {d.N}], got {tuple(t.shape)}")
        if t.shape[0] > d.max_slots:
            raise ValueError(f"{name}: {t.shape[0]} slots exceed max_slots={d.max_slots}")
        return int(t.shape[0])

    def _check_pilots(self, p: torch.Tensor):
        d = self.desc
        if (p.dtype != torch.complex64 or p.device.type != "cuda" or not p.is_contiguous()
                or tuple(p.shape) != (d.K, d.N)):
            raise ValueError(f"pilots must be a contiguous complex64 CUDA [{d.K}, {d.N}] tensor")

    def workspace_bytes(self, slots: int) -> int:
        return workspace_size(self.desc, slots)

    def _workspace(self, slots: int) -> tuple[ctypes.c_void_p, int]:
        need = self.workspace_bytes(slots)
        if need == 0:
            return ctypes.c_void_p(0), 0
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return _ptr(self._ws), int(self._ws.numel())

    # ---- design
    def set_design(self, tau_rms: float, sigma2: float, stream=None):
        check(self._lib.lmmse_set_design(self._h, float(tau_rms), float(sigma2), _stream_ptr(stream)),
              "lmmse_set_design")

    def set_filters(self, w: torch.Tensor, stream=None):
        d = self.desc
        if (w.dtype != torch.complex128 or w.device.type != "cuda" or not w.is_contiguous()
                or tuple(w.shape) != (self.n_classes, d.B, d.Wn)):
            raise ValueError(f"w must be a contiguous complex128 CUDA [{self.n_classes}, {d.B}, {d.Wn}] tensor")
        check(self._lib.lmmse_set_filters(self._h, _ptr(w), _stream_ptr(stream)), "lmmse_set_filters")

    def set_input_scale(self, scale: float):
        """Power-of-two scale of the LS values inside the split-precision
        filtering (undone on the output)."""
        check(self._lib.lmmse_set_input_scale(self._h, float(scale)), "lmmse_set_input_scale")

    def set_correlation(self, r: torch.Tensor, stream=None):
        """Caller correlation (rsource 'user_r'): r is a complex128 CUDA [N, N]
        Hermitian matrix; the plan designs one filter per block from it."""
        d = self.desc
        if (r.dtype != torch.complex128 or r.device.type != "cuda" or not r.is_contiguous()
                or tuple(r.shape) != (d.N, d.N)):
            raise ValueError(f"r must be a contiguous complex128 CUDA [{d.N}, {d.N}] tensor")
        check(self._lib.lmmse_set_correlation(self._h, _ptr(r), _stream_ptr(stream)),
              "lmmse_set_correlation")

    def get_filters(self, stream=None) -> torch.Tensor:
        d = self.desc
        w = torch.empty((self.n_classes, d.B, d.Wn), dtype=torch.complex128, device=self.device)
        check(self._lib.lmmse_get_filters(self._h, _ptr(w), _stream_ptr(stream)), "lmmse_get_filters")
        return w

    # ---- forward
    def despread(self, y, pilots, out=None, stream=None) -> torch.Tensor:
        S = self._check_cols(y, "y")
        self._check_pilots(pilots)
        out = torch.empty_like(y) if out is None else out
        self._check_cols(out, "out")
        check(self._lib.lmmse_despread(self._h, S, _ptr(y), _ptr(pilots), _ptr(out), _stream_ptr(stream)),
              "lmmse_despread")
        return out

    def apply(self, h_ls, out=None, stream=None) -> torch.Tensor:
        S = self._check_cols(h_ls, "h_ls")
        out = torch.empty_like(h_ls) if out is None else out
        self._check_cols(out, "out")
        check(self._lib.lmmse_apply(self._h, S, _ptr(h_ls), _ptr(out), _stream_ptr(stream)), "lmmse_apply")
        return out

    def covariance(self, h_ls, out=None, stream=None) -> torch.Tensor:
        S = self._check_cols(h_ls, "h_ls")
        d = self.desc
        shape = (S, d.K, self.nb, d.Wn, d.Wn)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        elif tuple(out.shape) != shape or out.dtype != torch.complex128 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex128 {shape} tensor")
        check(self._lib.lmmse_covariance(self._h, S, _ptr(h_ls), _ptr(out), _stream_ptr(stream)),
              "lmmse_covariance")
        return out

    def sample_filters(self, r_win, sigma2: float, out=None, stream=None) -> torch.Tensor:
        d = self.desc
        if r_win.dtype != torch.complex128 or r_win.dim() != 5 or not r_win.is_contiguous() \
                or tuple(r_win.shape[1:]) != (d.K, self.nb, d.Wn, d.Wn):
            raise ValueError("r_win must be a contiguous complex128 [S, K, N/B, Wn, Wn] tensor")
        S = int(r_win.shape[0])
        shape = (S, d.K, self.nb, d.B, d.Wn)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        b = ctypes.c_size_t(0)
        check(self._lib.lmmse_sample_filters_workspace_size(ctypes.byref(self.desc), S, ctypes.byref(b)),
              "lmmse_sample_filters_workspace_size")
        ws = torch.empty(b.value, dtype=torch.uint8, device=self.device) if b.value else None
        check(self._lib.lmmse_sample_filters(self._h, S, _ptr(r_win), float(sigma2), _ptr(out),
                                             _ptr(ws) if ws is not None else None, b.value,
                                             _stream_ptr(stream)), "lmmse_sample_filters")
        return out

    def estimate(self, y, pilots, sigma2: float, out=None, stream=None) -> torch.Tensor:
        """estimate(y_pilot, pilots, sigma2, block plan) -> h_hat."""
        S = self._check_cols(y, "y")
        self._check_pilots(pilots)
        out = torch.empty_like(y) if out is None else out
        self._check_cols(out, "out")
        ws, wsb = self._workspace(S)
        check(self._lib.lmmse_estimate(self._h, S, _ptr(y), _ptr(pilots), float(sigma2), _ptr(out),
                                       ws, wsb, _stream_ptr(stream)), "lmmse_estimate")
        return out

    def estimate_noalloc(self, y, pilots, sigma2: float, out=None, stream=None) -> torch.Tensor:
        """estimate() on the library's static device workspace (lmmse_estimate_noalloc):
        nothing is allocated by the library; `out` may be passed so that
        nothing is allocated here either."""
        S = self._check_cols(y, "y")
        self._check_pilots(pilots)
        out = torch.empty_like(y) if out is None else out
        self._check_cols(out, "out")
        check(self._lib.lmmse_estimate_noalloc(self._h, S, _ptr(y), _ptr(pilots), float(sigma2),
                                               _ptr(out), _stream_ptr(stream)),
              "lmmse_estimate_noalloc")
        return out

    def estimate_ls(self, h_ls, sigma2: float, out=None, stream=None, keep=None) -> torch.Tensor:
        """The estimator from LS estimates, h_ls -> h_hat (records sigma2 as the design noise).
        keep: a device uint8 tensor of design_state_bytes(S) bytes that receives the
        sample design for backward(..., kept=keep) (lmmse_estimate_ls_keep)."""
        S = self._check_cols(h_ls, "h_ls")
        out = torch.empty_like(h_ls) if out is None else out
        self._check_cols(out, "out")
        ws, wsb = self._workspace(S)
        if keep is not None:
            self._check_state(keep)
            check(self._lib.lmmse_estimate_ls_keep(self._h, S, _ptr(h_ls), float(sigma2), _ptr(out),
                                                   _ptr(keep), int(keep.numel()), ws, wsb,
                                                   _stream_ptr(stream)), "lmmse_estimate_ls_keep")
            return out
        check(self._lib.lmmse_estimate_ls(self._h, S, _ptr(h_ls), float(sigma2), _ptr(out), ws, wsb,
                                          _stream_ptr(stream)), "lmmse_estimate_ls")
        return out

    def design_state_bytes(self, slots: int) -> int:
        """Bytes of the sample design estimate_ls(..., keep=) keeps (0: not available)."""
        b = ctypes.c_size_t(0)
        check(self._lib.lmmse_design_state_size(self._h, int(slots), ctypes.byref(b)),
              "lmmse_design_state_size")
        return b.value

    @staticmethod
    def _check_state(t):
        if not t.is_cuda or t.dtype != torch.uint8 or not t.is_contiguous():
            raise ValueError("design state: contiguous device uint8 tensor")

    # ---- backward
    def backward(self, h_ls, g, want_params: bool = True, out=None, stream=None, params_out=None,
                 kept=None):
        """Returns (d_hls, d_tau, d_sigma2); the scalars are None unless requested.
        With params_out (a device float64 tensor of 2 elements) the scalars stay
        on the device (lmmse_backward_dev): params_out[0] and params_out[1] are
        returned as tensors and nothing waits for the host.  kept: the design
        state estimate_ls(h_ls, ..., keep=) filled for this h_ls
        (lmmse_backward_kept; needs params_out)."""
        S = self._check_cols(h_ls, "h_ls")
        self._check_cols(g, "g")
        if kept is not None and params_out is None:
            raise ValueError("kept: the kept-design backward leaves the scalars on the device; pass params_out")
        out = torch.empty_like(h_ls) if out is None else out
        ws, wsb = self._workspace(S)
        if params_out is not None:
            if (not params_out.is_cuda or params_out.dtype != torch.float64 or params_out.numel() < 2
                    or not params_out.is_contiguous()):
                raise ValueError("params_out: contiguous device float64 tensor of 2 elements")
            if kept is not None:
                self._check_state(kept)
                check(self._lib.lmmse_backward_kept(self._h, S, _ptr(h_ls), _ptr(g), _ptr(out),
                                                    _ptr(params_out), _ptr(kept), int(kept.numel()),
                                                    ws, wsb, _stream_ptr(stream)),
                      "lmmse_backward_kept")
                return out, params_out[0], params_out[1]
            check(self._lib.lmmse_backward_dev(self._h, S, _ptr(h_ls), _ptr(g), _ptr(out),
                                               _ptr(params_out), ws, wsb, _stream_ptr(stream)),
                  "lmmse_backward_dev")
            return out, params_out[0], params_out[1]
        dt = ctypes.c_double(math.nan)
        ds = ctypes.c_double(math.nan)
        check(self._lib.lmmse_backward(self._h, S, _ptr(h_ls), _ptr(g), _ptr(out),
                                       ctypes.byref(dt) if want_params else None,
                                       ctypes.byref(ds) if want_params else None,
                                       ws, wsb, _stream_ptr(stream)), "lmmse_backward")
        if want_params:
            return out, dt.value, ds.value
        return out, None, None

    def sync_status(self, stream=None):
        info = ctypes.c_int(-1)
        st = self._lib.lmmse_sync_status(self._h, _stream_ptr(stream), ctypes.byref(info))
        return st, info.value


_COMB_KIND = {"3w": _lib.COMB_3W, "12w": _lib.COMB_12W, "ls_hold": _lib.COMB_LS_HOLD,
              "ls_linear": _lib.COMB_LS_LINEAR, "ls_linear3": _lib.COMB_LS_LINEAR3,
              "ls_quadratic": _lib.COMB_LS_QUADRATIC, "ls_spline": _lib.COMB_LS_SPLINE}


def make_comb_desc(M, K, N, N_fft, comb=12, kind="12w", rsource="uniform", L=8.0, tau_rms=1.0,
                   taps=1, sigma2=0.1, max_slots=1) -> CombDesc:
    return CombDesc(M=int(M), K=int(K), comb=int(comb), N=int(N), N_fft=int(N_fft),
                    kind=_COMB_KIND[kind] if isinstance(kind, str) else int(kind),
                    rsource=_RSOURCE[rsource] if isinstance(rsource, str) else int(rsource),
                    taps=int(taps), tau_rms=float(tau_rms), L=float(L), sigma2=float(sigma2),
                    max_slots=int(max_slots))


def comb_validate(**kw) -> int:
    """Status of a comb descriptor (host only)."""
    d = make_comb_desc(**kw)
    return _lib.load().lmmse_comb_validate(ctypes.byref(d))


class CombPlan:
    """Comb-pilot 3W / 12W estimator on the current GPU (see include/lmmse.h)."""

    def __init__(self, **kw):
        self._lib = _lib.load()
        self.desc = make_comb_desc(**kw)
        h = ctypes.c_void_p()
        check(self._lib.lmmse_comb_create(ctypes.byref(self.desc), ctypes.byref(h)),
              "lmmse_comb_create")
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        d = self.desc
        self.win = {_lib.COMB_3W: 3, _lib.COMB_12W: 12}.get(d.kind, 1)
        self.nout = {_lib.COMB_3W: 3, _lib.COMB_12W: d.comb}.get(d.kind, 1)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.lmmse_comb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get_filters(self, stream=None) -> torch.Tensor:
        """FP64 filter classes, complex128 [K][win][nout][win]."""
        d = self.desc
        w = torch.empty((d.K, self.win, self.nout, self.win), dtype=torch.complex128, device=self.device)
        check(self._lib.lmmse_comb_get_filters(self._h, _ptr(w), _stream_ptr(stream)),
              "lmmse_comb_get_filters")
        return w

    def estimate(self, y, pilots, out=None, stream=None) -> torch.Tensor:
        """y: complex64 [S][M][N] comb pilot symbol; pilots: complex64 [N].
        Returns complex64 [S][M][K][N]."""
        d = self.desc
        if (y.dtype != torch.complex64 or y.device.type != "cuda" or not y.is_contiguous()
                or y.dim() != 3 or tuple(y.shape[1:]) != (d.M, d.N) or y.shape[0] > d.max_slots):
            raise ValueError(f"y must be a contiguous complex64 CUDA [S<={d.max_slots}, {d.M}, {d.N}] tensor")
        if (pilots.dtype != torch.complex64 or pilots.device.type != "cuda"
                or not pilots.is_contiguous() or tuple(pilots.shape) != (d.N,)):
            raise ValueError(f"pilots must be a contiguous complex64 CUDA [{d.N}] tensor")
        S = int(y.shape[0])
        shape = (S, d.M, d.K, d.N)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=y.device)
        elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex64 {shape} tensor")
        check(self._lib.lmmse_comb_estimate(self._h, S, _ptr(y), _ptr(pilots), _ptr(out),
                                            _stream_ptr(stream)), "lmmse_comb_estimate")
        return out


def mmse_detect(h_hat: torch.Tensor, y_data: torch.Tensor, sigma2: float, out=None,
                stream=None) -> torch.Tensor:
    """MMSE MIMO detection (eq. 22) per (slot, subcarrier).
    h_hat: complex64 [S, M, K, N]; y_data: complex64 [S, M, T, N].
    Returns complex64 [S, T, K, N]."""
    for t, name in ((h_hat, "h_hat"), (y_data, "y_data")):
        if t.dtype != torch.complex64 or t.device.type != "cuda" or not t.is_contiguous() or t.dim() != 4:
            raise ValueError(f"{name} must be a contiguous complex64 CUDA 4-d tensor")
    S, M, K, N = h_hat.shape
    if y_data.shape[0] != S or y_data.shape[1] != M or y_data.shape[3] != N:
        raise ValueError("y_data must be [S, M, T, N] matching h_hat")
    T = int(y_data.shape[2])
    shape = (S, T, K, N)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=h_hat.device)
    elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous complex64 {shape} tensor")
    lib = _lib.load()
    check(lib.lmmse_mmse_detect(int(S), int(M), int(K), T, int(N), _ptr(h_hat), _ptr(y_data),
                                float(sigma2), _ptr(out), _stream_ptr(stream)), "lmmse_mmse_detect")
    return out
