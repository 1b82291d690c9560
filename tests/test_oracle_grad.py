"""Pins of the oracle's hand-derived gradients: central finite differences in
FP64 (relative step 1e-4 on tau and sigma2, a random complex direction for
H_LS) and an independent PyTorch CPU complex128 autograd of the same loss."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import make_slot_batch

SMALL = dict(M=6, K=2, N=48, N_fft=64, taps=6, tau=3.0, snr_db=10.0)


def _fixed_loss(X, H, B, Wn, tau, taps, N_fft, sigma2, K):
    N = X.shape[-1]
    n = np.arange(N)
    R = O.toeplitz_from_r(lambda d: O.r_exponential(d, tau, taps, N_fft), n, n)
    Ws, st = O.block_filters(R, B, Wn, sigma2 / K)
    return O.mse_loss_and_grad(O.apply_filters(Ws, st, B, X), H)


def _sample_loss(X, H, B, Wn, sigma2):
    S, M, K, N = X.shape
    lam = sigma2 / K
    out = np.zeros_like(X)
    starts, offs = O.window_starts(N, B, Wn)
    for s in range(S):
        for k in range(K):
            for b, (st, off) in enumerate(zip(starts, offs)):
                Xw = X[s, :, k, st:st + Wn]
                R = O.sample_covariance(Xw)
                A = R + lam * np.eye(Wn)
                W = R[off:off + B] @ np.linalg.inv(A)
                out[s, :, k, b * B:(b + 1) * B] = Xw @ W.T
    return O.mse_loss_and_grad(out, H)


@pytest.fixture(scope="module")
def data():
    sb = make_slot_batch(**SMALL, slots=2)
    X = O.despread(sb.y, sb.pilots)
    return sb, X


@pytest.mark.parametrize("B,Wn", [(8, 8), (8, 16), (48, 48)])
def test_fixed_design_grad_vs_finite_differences(data, B, Wn):
    sb, X = data
    K, tau, sig2 = 2, 4.5, 0.02
    args = (B, Wn, tau, 6, 64, sig2, K)
    L0, G = _fixed_loss(X, sb.H, *args)
    dX, gtau, gsig = O.grad_fixed_design(X, G, B, Wn, tau, 6, 64, sig2, K)
    h = 1e-4
    fd_tau = (_fixed_loss(X, sb.H, B, Wn, tau * (1 + h), 6, 64, sig2, K)[0]
              - _fixed_loss(X, sb.H, B, Wn, tau * (1 - h), 6, 64, sig2, K)[0]) / (2 * h * tau)
    fd_sig = (_fixed_loss(X, sb.H, B, Wn, tau, 6, 64, sig2 * (1 + h), K)[0]
              - _fixed_loss(X, sb.H, B, Wn, tau, 6, 64, sig2 * (1 - h), K)[0]) / (2 * h * sig2)
    assert abs(gtau - fd_tau) <= 1e-6 * abs(fd_tau) + 1e-12
    assert abs(gsig - fd_sig) <= 1e-6 * abs(fd_sig) + 1e-12
    rng = np.random.default_rng(0)
    V = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
    V /= np.linalg.norm(V)
    e = 1e-4
    fd_x = (_fixed_loss(X + e * V, sb.H, *args)[0] - _fixed_loss(X - e * V, sb.H, *args)[0]) / (2 * e)
    an_x = float(np.sum(np.conj(dX) * V).real)
    assert abs(an_x - fd_x) <= 1e-6 * abs(fd_x) + 1e-12


def test_sample_cov_grad_vs_finite_differences(data):
    sb, X = data
    B, Wn, sig2 = 8, 16, 0.02
    L0, G = _sample_loss(X, sb.H, B, Wn, sig2)
    dX, gsig = O.grad_sample_cov(X, G, B, Wn, sig2)
    h = 1e-4
    fd_sig = (_sample_loss(X, sb.H, B, Wn, sig2 * (1 + h))[0]
              - _sample_loss(X, sb.H, B, Wn, sig2 * (1 - h))[0]) / (2 * h * sig2)
    assert abs(gsig - fd_sig) <= 1e-6 * abs(fd_sig) + 1e-12
    rng = np.random.default_rng(1)
    V = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
    V /= np.linalg.norm(V)
    e = 1e-5
    fd_x = (_sample_loss(X + e * V, sb.H, B, Wn, sig2)[0] - _sample_loss(X - e * V, sb.H, B, Wn, sig2)[0]) / (2 * e)
    an_x = float(np.sum(np.conj(dX) * V).real)
    assert abs(an_x - fd_x) <= 1e-5 * abs(fd_x) + 1e-12
    # the fixed-design formula W^H G alone is not the gradient here
    Wonly = np.zeros_like(X)
    assert np.linalg.norm(dX) > 0 and not np.allclose(dX, Wonly)


def _torch_fixed(Xn, Hn, B, Wn, taps, N_fft, K, tau0, sig0):
    X = torch.tensor(Xn, dtype=torch.complex128, requires_grad=True)
    H = torch.tensor(Hn, dtype=torch.complex128)
    tau = torch.tensor(tau0, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(sig0, dtype=torch.float64, requires_grad=True)
    N = X.shape[-1]
    l = torch.arange(taps, dtype=torch.float64)
    w = torch.exp(-l / tau)
    p = w / w.sum()
    n = torch.arange(N, dtype=torch.float64)
    d = n[:, None] - n[None, :]
    ph = torch.exp(-2j * torch.pi * d[..., None] * l / N_fft)
    R = (ph * p.to(torch.complex128)).sum(-1)
    lam = sig / K
    outs = []
    starts, _ = O.window_starts(N, B, Wn)   # integer plan only
    for b, s in enumerate(starts):
        Rii = R[s:s + Wn, s:s + Wn]
        Rio = R[s:s + Wn, b * B:(b + 1) * B]
        A = Rii + lam * torch.eye(Wn, dtype=torch.complex128)
        Lc = torch.linalg.cholesky(A)
        WH = torch.cholesky_solve(Rio, Lc)           # A^-1 R_IO = W^H
        outs.append(X[..., s:s + Wn] @ WH.conj())    # rows: (W x)^T = x^T W^T
    out = torch.cat(outs, dim=-1)
    loss = (out - H).abs().pow(2).sum() / out.numel()
    loss.backward()
    return float(loss.detach()), X.grad.numpy(), float(tau.grad), float(sig.grad)


@pytest.mark.parametrize("B,Wn", [(8, 16), (16, 16)])
def test_fixed_design_grad_vs_torch_autograd(data, B, Wn):
    sb, X = data
    K, tau, sig2 = 2, 4.5, 0.02
    L0, G = _fixed_loss(X, sb.H, B, Wn, tau, 6, 64, sig2, K)
    dX, gtau, gsig = O.grad_fixed_design(X, G, B, Wn, tau, 6, 64, sig2, K)
    lt, dXt, gtau_t, gsig_t = _torch_fixed(X, sb.H, B, Wn, 6, 64, K, tau, sig2)
    assert abs(lt - L0) < 1e-12 * abs(L0) + 1e-15
    np.testing.assert_allclose(dX, dXt, rtol=1e-9, atol=1e-13)
    assert abs(gtau - gtau_t) <= 1e-9 * abs(gtau_t) + 1e-15
    assert abs(gsig - gsig_t) <= 1e-9 * abs(gsig_t) + 1e-15


def test_dr_dtau_vs_finite_differences():
    d = np.arange(-80, 81)
    for tau in (2.0, 8.0, 24.0):
        h = 1e-5 * tau
        fd = (O.r_exponential(d, tau + h, 72, 2048) - O.r_exponential(d, tau - h, 72, 2048)) / (2 * h)
        np.testing.assert_allclose(O.dr_exponential_dtau(d, tau, 72, 2048), fd, atol=1e-9)


def test_expected_mse_stationary_at_truth():
    # The exponential family contains the matched design: the expected error
    # of the partitioned estimator is stationary in (tau, sigma2) at the truth.
    N, K, N_fft, taps, tau0, sig0 = 96, 4, 256, 16, 3.0, 0.1
    n = np.arange(N)
    Rt = O.toeplitz_from_r(lambda d: O.r_exponential(d, tau0, taps, N_fft), n, n)

    def emse(tau, sig):
        R = O.toeplitz_from_r(lambda d: O.r_exponential(d, tau, taps, N_fft), n, n)
        Ws, st = O.block_filters(R, 12, 36, sig / K)
        return O.expected_mse(Rt, sig0 / K, Ws, st, 12)

    h = 1e-4
    gt = (emse(tau0 * (1 + h), sig0) - emse(tau0 * (1 - h), sig0)) / (2 * h * tau0)
    gs = (emse(tau0, sig0 * (1 + h)) - emse(tau0, sig0 * (1 - h))) / (2 * h * sig0)
    # compare with the sensitivity away from the truth
    ga = (emse(2 * tau0 * (1 + h), sig0) - emse(2 * tau0 * (1 - h), sig0)) / (4 * h * tau0)
    assert abs(gt) < 1e-6 * abs(ga) + 1e-12
    assert abs(gs) < 1e-5
