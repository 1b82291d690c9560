"""FP64 oracle of MMSE MIMO detection (Sec. IV-A, MMSE MIMO detector, eq. 20-22).  Test
infrastructure only, like the rest of this package.

Per (slot, data subcarrier n) with H the M x K channel estimate and Y the
M x T received data symbols, the detected symbols solve
    (H^H H + sigma2 I) X = H^H Y                                   (eq. 22)
with the Hermitian positive definite system factored by Cholesky (the
paper's LAPACKE_cposv route).  sigma2 is the receive noise variance per
resource element with unit-power symbols.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .lmmse import C128


def mmse_detect(H, Y, sigma2: float) -> np.ndarray:
    """H: [S][M][K][N] channel (estimate); Y: [S][M][T][N] received data
    symbols.  Returns X [S][T][K][N] complex128 solving eq. 22 per (s, n)."""
    H = np.asarray(H).astype(C128)
    Y = np.asarray(Y).astype(C128)
    S, M, K, N = H.shape
    T = Y.shape[2]
    X = np.zeros((S, T, K, N), dtype=C128)
    for s in range(S):
        for n in range(N):
            h = H[s, :, :, n]                      # M x K
            A = np.conj(h).T @ h + float(sigma2) * np.eye(K)
            b = np.conj(h).T @ Y[s, :, :, n]        # K x T
            X[s, :, :, n] = sla.cho_solve(sla.cho_factor(A, lower=True), b).T
    return X


def qpsk_decide(x) -> np.ndarray:
    """Nearest unit-power QPSK point of each symbol."""
    x = np.asarray(x)
    return (np.sign(x.real) + 1j * np.sign(x.imag)) / np.sqrt(2.0)
