"""FP64 optimum of the fixed-design fit (test infrastructure only).

The paper picks the assumed channel length of its fixed design (eq. 16 /
eq. 17) by measured BER (Sec. IV-C).  The gradient fit replaces that choice:
it tunes the assumed (tau_rms, sigma2) of the exponential design by
minimising the simulated MSE of the partitioned estimator when the channels'
delay spread is itself random, tau ~ U[lo, hi] per (slot, user).  This module
gives the target of that fit without any simulation:

  * The expected squared error of a linear estimator is linear in the true
    channel correlation (expected_mse: tr(R_OO - W R_IO - R_OI W^H +
    W (R_II + lam I) W^H)), so averaging it over the delay spread equals
    evaluating it once at the averaged correlation
        rbar_d = E_tau[r_d(tau)] = (1 / (hi - lo)) int_lo^hi r_d(tau) dtau,
    which is computed here by Gauss-Legendre quadrature over tau.
  * The optimum (tau*, sigma2*) minimises that expected error over the two
    design parameters (Nelder-Mead on their logarithms, FP64 throughout).

With lo == hi the averaged correlation is the single-spread one and the
optimum is the truth (the exponential family contains the matched filters).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize as sopt

from .lmmse import block_filters, expected_mse, r_exponential, toeplitz_from_r


def mixture_r(d, tau_lo: float, tau_hi: float, taps: int, N_fft: int, nodes: int = 48) -> np.ndarray:
    """rbar_d = E[r_d(tau)] for tau ~ U[tau_lo, tau_hi] (r_d the discrete
    exponential tap sum), by `nodes`-point Gauss-Legendre quadrature; the
    single-spread r_d when tau_lo == tau_hi."""
    d = np.asarray(d, dtype=np.float64)
    lo, hi = float(tau_lo), float(tau_hi)
    if hi == lo:
        return r_exponential(d, lo, taps, N_fft)
    x, w = np.polynomial.legendre.leggauss(int(nodes))
    taus = 0.5 * (hi - lo) * x + 0.5 * (hi + lo)
    acc = np.zeros(d.shape, dtype=np.complex128)
    for t, wt in zip(taus, w):
        acc += 0.5 * wt * r_exponential(d, t, taps, N_fft)   # weights sum to 2
    return acc


def design_mse(tau_d: float, sigma2_d: float, R_true: np.ndarray, lam_true: float,
               B: int, Wn: int, K: int, taps: int, N_fft: int) -> float:
    """Expected error per coefficient of the partitioned estimator designed
    with the exponential r_d(tau_d) and lam = sigma2_d / K, on channels of
    correlation R_true with LS noise variance lam_true."""
    N = R_true.shape[0]
    n = np.arange(N)
    R_d = toeplitz_from_r(lambda dd: r_exponential(dd, tau_d, taps, N_fft), n, n)
    Ws, starts = block_filters(R_d, B, Wn, float(sigma2_d) / K)
    return expected_mse(R_true, lam_true, Ws, starts, B)


def fit_optimum(N: int, B: int, Wn: int, K: int, taps: int, N_fft: int, sigma2_true: float,
                tau_lo: float, tau_hi: float, x0=(8.0, 1e-2), xatol: float = 1e-7,
                fatol: float = 1e-15):
    """Minimiser of the expected error over the design (tau, sigma2) for
    channels with tau ~ U[tau_lo, tau_hi] and noise variance sigma2_true per
    resource element (LS noise sigma2_true / K).  Returns
    (tau*, sigma2*, mse*, R_bar)."""
    n = np.arange(N)
    R_bar = toeplitz_from_r(lambda d: mixture_r(d, tau_lo, tau_hi, taps, N_fft), n, n)
    lam_true = float(sigma2_true) / K

    def f(z):
        return design_mse(float(np.exp(z[0])), float(np.exp(z[1])), R_bar, lam_true, B, Wn, K,
                          taps, N_fft)

    z0 = np.log(np.asarray(x0, dtype=np.float64))
    res = sopt.minimize(f, z0, method="Nelder-Mead",
                        options=dict(xatol=xatol, fatol=fatol, maxiter=4000, maxfev=8000))
    tau_s, sig_s = float(np.exp(res.x[0])), float(np.exp(res.x[1]))
    return tau_s, sig_s, float(res.fun), R_bar
