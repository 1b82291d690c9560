"""Pins of the oracle's fit optimum (oracle/fit_optimum.py), CPU only.

The optimum of the fixed-design fit over channels with a random delay spread
has no closed form.  It is pinned by what fixes it independently:
  * the averaged correlation against a dense midpoint rule and against the
    empirical covariance of the slot generator (which draws tau per user);
  * linearity of the expected error in the true correlation, checked by
    brute-force averaging over channel draws' correlations;
  * single-spread data, where the optimum is the truth;
  * a grid search and a finite-difference stationarity check around it;
  * the stored optimum of the differentiation workload, recomputed.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle.fit_optimum import design_mse, fit_optimum, mixture_r
from synth import make_slot_batch


def test_mixture_r_single_spread_and_narrow_interval():
    d = np.arange(-60, 61)
    np.testing.assert_allclose(mixture_r(d, 5.0, 5.0, 72, 2048), O.r_exponential(d, 5.0, 72, 2048),
                               rtol=0, atol=0)
    np.testing.assert_allclose(mixture_r(d, 5.0, 5.0 + 1e-7, 72, 2048),
                               O.r_exponential(d, 5.0 + 5e-8, 72, 2048), atol=1e-12)


def test_mixture_r_matches_dense_midpoint_rule():
    d = np.arange(-150, 151)
    lo, hi, P = 2.0, 24.0, 20000
    mids = lo + (np.arange(P) + 0.5) * (hi - lo) / P
    ref = np.zeros(d.shape, dtype=np.complex128)
    for t in mids:
        ref += O.r_exponential(d, t, 72, 2048)
    ref /= P
    np.testing.assert_allclose(mixture_r(d, lo, hi, 72, 2048), ref, atol=1e-8)


def test_mixture_r_matches_generator_with_random_spread():
    # channels drawn with tau ~ U[2, 24] per (slot, user) by the slot generator
    sb = make_slot_batch(M=64, K=4, N=40, N_fft=256, taps=40, tau=(2.0, 24.0), snr_db=None,
                         slots=24, config_id=91, noiseless=True)
    H = sb.H.transpose(0, 1, 2, 3).reshape(-1, 40)          # every (slot, antenna, user)
    emp = (H[:, :, None] * np.conj(H[:, None, :])).mean(axis=0)
    n = np.arange(40)
    Rb = O.toeplitz_from_r(lambda d: mixture_r(d, 2.0, 24.0, 40, 256), n, n)
    # 24 slots x 4 users = 96 spread draws: the statistical error of the
    # entries is about 1/sqrt(96 * 64)^(1/2) at worst; the bar is loose on it
    assert np.max(np.abs(emp - Rb)) < 0.08
    assert np.linalg.norm(emp - Rb) / np.linalg.norm(Rb) < 0.05


def test_expected_error_is_linear_in_the_true_correlation():
    # averaging the error over spreads equals the error at the averaged R
    N, B, Wn, K, taps, N_fft = 48, 12, 20, 4, 24, 256
    n = np.arange(N)
    taus = [2.0, 5.0, 11.0]
    Rs = [O.toeplitz_from_r(lambda d, t=t: O.r_exponential(d, t, taps, N_fft), n, n) for t in taus]
    avg = np.mean([design_mse(6.0, 0.05, R, 0.1 / K, B, Wn, K, taps, N_fft) for R in Rs])
    at_mean = design_mse(6.0, 0.05, sum(Rs) / 3, 0.1 / K, B, Wn, K, taps, N_fft)
    assert abs(avg - at_mean) < 1e-14


def test_design_mse_matches_monte_carlo_of_the_estimator():
    # the expected error of the designed filters against brute-force
    # estimation on drawn slots (independent route: generator + oracle)
    N, B, Wn, K, taps, N_fft, sig = 48, 12, 24, 2, 16, 128, 0.1
    sb = make_slot_batch(M=64, K=K, N=N, N_fft=N_fft, taps=taps, tau=3.0, snr_db=10.0, slots=8,
                         config_id=92)
    out = O.estimate(sb.y, sb.pilots, sb.sigma2, B, Wn, "exp", N_fft=N_fft, tau=6.0, taps=taps)
    mc = float(np.mean(np.abs(out - sb.H) ** 2))
    n = np.arange(N)
    Rt = O.toeplitz_from_r(lambda d: O.r_exponential(d, 3.0, taps, N_fft), n, n)
    ex = design_mse(6.0, sb.sigma2, Rt, sb.sigma2 / K, B, Wn, K, taps, N_fft)
    assert abs(mc - ex) / ex < 0.06


def test_fit_optimum_single_spread_is_the_truth():
    tau, sig, mse, _ = fit_optimum(96, 12, 36, 4, 16, 256, 0.1, 3.0, 3.0, x0=(8.0, 1e-2))
    assert abs(tau - 3.0) / 3.0 < 1e-5
    assert abs(sig - 0.1) / 0.1 < 1e-4


def test_fit_optimum_random_spread_beats_grid_and_is_stationary():
    N, B, Wn, K, taps, N_fft, sig0 = 96, 12, 36, 4, 24, 256, 0.1
    tau, sig, mse, Rb = fit_optimum(N, B, Wn, K, taps, N_fft, sig0, 2.0, 12.0)
    lam = sig0 / K
    f = lambda t, s: design_mse(t, s, Rb, lam, B, Wn, K, taps, N_fft)  # noqa: E731
    grid = [f(t, s) for t in np.geomspace(1.5, 14.0, 9) for s in np.geomspace(1e-3, 1.0, 9)]
    assert mse <= min(grid) + 1e-15
    h = 1e-4
    gt = (f(tau * (1 + h), sig) - f(tau * (1 - h), sig)) / (2 * h)
    gs = (f(tau, sig * (1 + h)) - f(tau, sig * (1 - h))) / (2 * h)
    # logarithmic sensitivities at twice the optimum for scale
    ga = (f(2 * tau * (1 + h), sig) - f(2 * tau * (1 - h), sig)) / (2 * h)
    assert abs(gt) < 1e-4 * abs(ga)
    assert abs(gs) < 1e-4 * abs(ga)
    # the spread mixture is not in the exponential family: the optimum is
    # strictly inside the interval and not the truth's noise
    assert 2.0 < tau < 12.0


@pytest.mark.slow
def test_stored_differentiation_workload_optimum(golden_dir):
    with open(os.path.join(golden_dir, "fit_optimum_diff_workload.json")) as f:
        g = json.load(f)
    c = g["config"]
    tau, sig, mse, _ = fit_optimum(c["N"], c["B"], c["Wn"], c["K"], c["taps"], c["N_fft"],
                                   c["sigma2"], c["tau_lo"], c["tau_hi"])
    assert abs(tau - g["tau"]) / g["tau"] < 1e-5
    assert abs(sig - g["sigma2"]) / g["sigma2"] < 1e-4
    assert abs(mse - g["mse"]) / g["mse"] < 1e-10
