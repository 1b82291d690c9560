"""FP64 oracle of the backward path (test infrastructure only).

The paper does not differentiate its estimator; it picks the assumed channel
length by measured BER (Sec. IV-C).  Here the partitioned estimator is made
differentiable in its inputs and in the design parameters, and this module
gives the hand-derived gradients in FP64, written out block by block.

Convention: for a real loss L and a complex array z, grad(z) = dL/dRe z +
j dL/dIm z, so that dL = Re sum conj(grad(z)) dz (the convention of PyTorch).
For one block with A = R_II + lam I, W = R_OI A^-1 and Hhat_O = W X_I:
    grad X_I   += W^H G_O
    grad W      = G_O X_I^H            (summed over columns)
    Z           = grad W  A^-1
    grad R_OI   = Z,   grad A = -W^H Z
    grad lam   += Re tr(grad A)
    grad tau   += Re sum conj(grad R_ij) dr(d_ij)/dtau   (R_ij = r(d_ij))
For a sample covariance R = X X^H / M of the window itself, X also receives
(Gam + Gam^H) X / M, with Gam the window-sized gradient of R.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .lmmse import C128, r_exponential, sample_covariance, toeplitz_from_r, window_starts


def dr_exponential_dtau(d, tau: float, taps: int, N_fft: int) -> np.ndarray:
    """d r_d / d tau for the discrete exponential profile p_l = e^{-l/tau}/S:
    dp_l/dtau = p_l (l - sum_i i p_i) / tau^2."""
    d = np.asarray(d, dtype=np.float64)
    l = np.arange(int(taps), dtype=np.float64)
    w = np.exp(-l / float(tau))
    p = w / w.sum()
    lbar = float((l * p).sum())
    dp = p * (l - lbar) / float(tau) ** 2
    ph = np.exp(-2j * np.pi * np.multiply.outer(d, l) / float(N_fft))
    return (ph * dp).sum(axis=-1)


def mse_loss_and_grad(H_hat, H_true):
    """L = sum |Hhat - H|^2 / n and its gradient 2 (Hhat - H) / n."""
    H_hat = np.asarray(H_hat).astype(C128)
    H_true = np.asarray(H_true).astype(C128)
    n = H_hat.size
    diff = H_hat - H_true
    return float(np.sum(np.abs(diff) ** 2) / n), 2.0 * diff / n


def _solve_right(A, dW):
    """dW A^-1 for Hermitian positive definite A (Cholesky)."""
    cf = sla.cho_factor(A, lower=True)
    return np.conj(sla.cho_solve(cf, np.conj(dW).T)).T


def grad_fixed_design(X, G, B: int, Wn: int, tau: float, taps: int, N_fft: int,
                      sigma2: float, K: int):
    """Gradients of the fixed exponential design estimator.

    X: H_LS [..., N]; G: grad wrt Hhat [..., N]; the filters come from the
    discrete exponential r_d(tau) and lam = sigma2 / K.
    Returns (grad X, grad tau, grad sigma2).
    """
    X = np.asarray(X).astype(C128)
    G = np.asarray(G).astype(C128)
    N = X.shape[-1]
    lam = float(sigma2) / K
    Xc = X.reshape(-1, N)
    Gc = G.reshape(-1, N)
    dX = np.zeros_like(Xc)
    n = np.arange(N)
    R = toeplitz_from_r(lambda d: r_exponential(d, tau, taps, N_fft), n, n)
    dR = toeplitz_from_r(lambda d: dr_exponential_dtau(d, tau, taps, N_fft), n, n)
    starts, _ = window_starts(N, B, Wn)
    g_tau = 0.0
    g_lam = 0.0
    for b, s in enumerate(starts):
        I = np.arange(s, s + Wn)
        O = np.arange(b * B, (b + 1) * B)
        A = R[np.ix_(I, I)] + lam * np.eye(Wn)
        W = _solve_right(A, R[np.ix_(O, I)])
        XI = Xc[:, I]                       # ncols x Wn
        GO = Gc[:, O]                       # ncols x B
        dX[:, I] += GO @ np.conj(W)         # (W^H G_O) per column
        dW = GO.T @ np.conj(XI)             # B x Wn
        Z = _solve_right(A, dW)
        gA = -np.conj(W).T @ Z
        g_lam += float(np.trace(gA).real)
        g_tau += float(np.sum(np.conj(Z) * dR[np.ix_(O, I)]).real)
        g_tau += float(np.sum(np.conj(gA) * dR[np.ix_(I, I)]).real)
    return dX.reshape(X.shape), g_tau, g_lam / K


def grad_sample_cov(X, G, B: int, Wn: int, sigma2: float):
    """Gradients of the sample-covariance estimator (per slot, user, window).

    X: H_LS [S][M][K][N]; G: grad wrt Hhat.  Returns (grad X, grad sigma2).
    """
    X = np.asarray(X).astype(C128)
    G = np.asarray(G).astype(C128)
    S, M, K, N = X.shape
    lam = float(sigma2) / K
    dX = np.zeros_like(X)
    starts, offs = window_starts(N, B, Wn)
    g_lam = 0.0
    for s in range(S):
        for k in range(K):
            for b, (st, off) in enumerate(zip(starts, offs)):
                Xw = X[s, :, k, st:st + Wn].T           # Wn x M
                R = sample_covariance(Xw.T)
                A = R + lam * np.eye(Wn)
                W = _solve_right(A, R[off:off + B, :])
                GO = G[s, :, k, b * B:(b + 1) * B].T    # B x M
                dXw = np.conj(W).T @ GO
                dW = GO @ np.conj(Xw).T
                Z = _solve_right(A, dW)
                gam = -np.conj(W).T @ Z
                g_lam += float(np.trace(gam).real)
                gam[off:off + B, :] += Z
                dXw += (gam + np.conj(gam).T) @ Xw / M
                dX[s, :, k, st:st + Wn] += dXw.T
    return dX, g_lam / K
