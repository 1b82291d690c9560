"""Pins of the FP64 oracle's forward path against things other than itself:
the paper's printed tables, closed forms, special cases, library routines on
a different route, brute force and Monte Carlo statistics."""
import os

import numpy as np
import pytest
import scipy.integrate as si

import oracle as O
from synth import exponential_pdp, make_slot_batch

TINY = dict(M=8, K=2, N=72, N_fft=128, taps=8, tau=2.0, snr_db=10.0)


# ------------------------------------------------------------------ pilots / LS
def test_cover_code_is_dft_and_orthogonal():
    for K in (1, 2, 3, 12, 24):
        c = O.cover_code(K)
        # the same matrix as numpy's DFT of the identity (a library route)
        np.testing.assert_allclose(c, np.fft.fft(np.eye(K), axis=0), atol=1e-12)
        np.testing.assert_allclose(np.conj(c) @ c.T / K, np.eye(K), atol=1e-12)


def test_despread_noiseless_recovers_channel():
    sb = make_slot_batch(**TINY, slots=2, noiseless=True)
    hls = O.despread(sb.y, sb.pilots)
    # y is complex64, so agreement is at single-precision rounding level
    assert O.nmse(hls, sb.H) < 1e-13


def test_despread_noiseless_paper_shape_user_isolation():
    # K = 12 with channels for only one user: the others must come out zero
    sb = make_slot_batch(M=2, K=12, N=48, N_fft=64, taps=4, tau=2.0, snr_db=None,
                         noiseless=True, slots=1)
    hls = O.despread(sb.y, sb.pilots)
    np.testing.assert_allclose(hls, sb.H, atol=2e-6)


def test_despread_noise_variance_is_sigma2_over_K():
    rng = np.random.default_rng(5)
    K, M, N, sigma2 = 4, 64, 256, 0.3
    w = (rng.standard_normal((1, M, K, N)) + 1j * rng.standard_normal((1, M, K, N))) * np.sqrt(sigma2 / 2)
    pil = np.exp(1j * np.pi / 4 * (2 * rng.integers(0, 4, (K, N)) + 1))
    z = O.despread(w, pil)
    v = np.mean(np.abs(z) ** 2)
    n = z.size
    assert abs(v - sigma2 / K) < 4 * (sigma2 / K) / np.sqrt(n)


# ------------------------------------------------------------------ correlation
def test_r_uniform_matches_quadrature_of_uniform_profile():
    L, N_fft = 144.0, 2048
    for d in (1, 3, 17, 100, -9):
        re = si.quad(lambda x: np.cos(2 * np.pi * x * d / N_fft), 0, L)[0] / L
        im = si.quad(lambda x: -np.sin(2 * np.pi * x * d / N_fft), 0, L)[0] / L
        np.testing.assert_allclose(O.r_uniform(d, L, N_fft), re + 1j * im, atol=1e-12)


def test_r_uniform_special_values():
    L, N_fft = 144.0, 2048
    assert O.r_uniform(0, L, N_fft) == 1.0
    # L d / N_fft = 9 d / 128 is a nonzero integer at d = 128: zero correlation
    assert abs(O.r_uniform(128, L, N_fft)) < 1e-15
    d = np.arange(-40, 41)
    np.testing.assert_allclose(O.r_uniform(-d, L, N_fft), np.conj(O.r_uniform(d, L, N_fft)), atol=1e-15)


def test_r_exponential_geometric_closed_form():
    for tau, taps, N_fft in ((2.0, 8, 128), (4.0, 72, 2048), (16.0, 72, 2048), (32.0, 144, 4096)):
        a = np.exp(-1.0 / tau)
        d = np.arange(-60, 61)
        q = a * np.exp(-2j * np.pi * d / N_fft)
        closed = (1 - a) / (1 - a ** taps) * (1 - q ** taps) / (1 - q)
        np.testing.assert_allclose(O.r_exponential(d, tau, taps, N_fft), closed, rtol=1e-12, atol=1e-14)


def test_r_exponential_matches_generator_statistics():
    # empirical E{H(a) H(b)^*} of the generator's channels
    sb = make_slot_batch(M=64, K=2, N=40, N_fft=128, taps=8, tau=2.0, snr_db=None,
                         noiseless=True, slots=8)
    Hc = sb.H.reshape(-1, 40)
    emp = (Hc[:, :, None] * np.conj(Hc[:, None, :])).mean(axis=0)
    n = np.arange(40)
    R = O.toeplitz_from_r(lambda d: O.r_exponential(d, 2.0, 8, 128), n, n)
    assert np.max(np.abs(emp - R)) < 5.0 / np.sqrt(Hc.shape[0])


def test_continuous_exponential_tends_to_uniform():
    d = np.arange(-30, 31)
    np.testing.assert_allclose(O.r_exponential_cont(d, 1e9, 144.0, 2048),
                               O.r_uniform(d, 144.0, 2048), atol=1e-6)


def test_toeplitz_hermitian_psd():
    n = np.arange(150)
    for R in (O.toeplitz_from_r(lambda d: O.r_uniform(d, 144, 2048), n, n),
              O.toeplitz_from_r(lambda d: O.r_exponential(d, 4.0, 72, 2048), n, n)):
        np.testing.assert_allclose(R, np.conj(R.T), atol=1e-15)
        assert np.linalg.eigvalsh(R).min() > -1e-10


# ------------------------------------------------------------------ block plan
def _parse_range(tok):
    tok = tok.strip()
    if ":" in tok:
        a, s, b = (int(v) for v in tok.split(":"))
        return list(range(a, b + 1, s))
    return [int(v) for v in tok.split(",")]


def _load_table(path):
    rows = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        idx, out, wid, ls = line.split(";")
        rows[int(idx)] = (_parse_range(out), int(wid), _parse_range(ls))
    return rows


@pytest.mark.parametrize("kind,fname", [("3w", "paper_table1_3w.txt"), ("12w", "paper_table2_12w.txt")])
def test_clamp_rule_reproduces_paper_tables(golden_dir, kind, fname):
    gold = _load_table(os.path.join(golden_dir, fname))
    table = {r[0]: r[1:] for r in O.comb_group_table(1200, 12, 1, kind)}
    assert len(table) == 100
    for idx, (out, wid, ls) in gold.items():
        assert table[idx][0] == out, idx
        assert table[idx][1] == wid, idx
        assert table[idx][2] == ls, idx
    # 3 distinct filters for 3W, 12 for 12W (Sec. IV-B)
    assert len({v[1] for v in table.values()}) == (3 if kind == "3w" else 12)


def test_window_starts_paper_sizes():
    s, off = O.window_starts(1200, 100, 150)
    assert s == [0] + [75 + 100 * i for i in range(10)] + [1050]
    assert sorted(set(off)) == [0, 25, 50]
    s, off = O.window_starts(3300, 132, 198)
    assert sorted(set(off)) == [0, 33, 66]
    s, off = O.window_starts(72, 12, 12)
    assert s == list(range(0, 72, 12)) and set(off) == {0}
    assert O.window_starts(1200, 1200, 1200) == ([0], [0])


def test_window_contains_output_block():
    rng = np.random.default_rng(1)
    for _ in range(200):
        B = int(rng.integers(1, 40))
        nb = int(rng.integers(1, 30))
        N = B * nb
        Wn = B + 2 * int(rng.integers(0, (N - B) // 2 + 1))
        s, off = O.window_starts(N, B, Wn)
        for b in range(nb):
            assert 0 <= s[b] <= b * B and b * B + B <= s[b] + Wn <= N


# ------------------------------------------------------------------ filters
def _R_exp(N, tau=2.0, taps=8, N_fft=128):
    n = np.arange(N)
    return O.toeplitz_from_r(lambda d: O.r_exponential(d, tau, taps, N_fft), n, n)


def test_single_block_equals_full_lmmse():
    R = _R_exp(72)
    Ws, starts = O.block_filters(R, 72, 72, 0.05)
    np.testing.assert_allclose(Ws[0], O.full_lmmse_filter(R, 0.05), atol=1e-12)
    # and the full filter satisfies the normal equations W (R + lam I) = R
    W = Ws[0]
    np.testing.assert_allclose(W @ (R + 0.05 * np.eye(72)), R, atol=1e-10)


def test_identity_correlation():
    R = np.eye(60, dtype=complex)
    for B, Wn in ((12, 12), (12, 36), (60, 60)):
        Ws, _ = O.block_filters(R, B, Wn, 0.25)
        for b, W in enumerate(Ws):
            _, off = O.window_starts(60, B, Wn)
            E = np.zeros((B, Wn))
            E[np.arange(B), off[b] + np.arange(B)] = 1
            np.testing.assert_allclose(W, E / 1.25, atol=1e-14)


def test_rank_one_correlation_sherman_morrison():
    N, lam = 48, 0.3
    R = np.ones((N, N), dtype=complex)
    for B, Wn in ((8, 8), (8, 24), (48, 48)):
        Ws, _ = O.block_filters(R, B, Wn, lam)
        for W in Ws:
            np.testing.assert_allclose(W, np.ones((B, Wn)) / (Wn + lam), atol=1e-12)


def test_vanishing_and_huge_noise_limits():
    R = _R_exp(36, tau=8.0, taps=36, N_fft=36)   # full rank Toeplitz
    Ws, starts = O.block_filters(R, 12, 24, 1e-10)
    _, off = O.window_starts(36, 12, 24)
    for b, W in enumerate(Ws):
        E = np.zeros((12, 24))
        E[np.arange(12), off[b] + np.arange(12)] = 1
        np.testing.assert_allclose(W, E, atol=1e-5)
    Ws, _ = O.block_filters(R, 12, 24, 1e10)
    assert max(np.abs(W).max() for W in Ws) < 1e-9


def test_fixed_design_has_at_most_three_filter_classes():
    n = np.arange(1200)
    R = O.toeplitz_from_r(lambda d: O.r_uniform(d, 144, 2048), n, n)
    Ws, starts = O.block_filters(R, 100, 150, 0.1 / 12)
    distinct = []
    for W in Ws:
        if not any(np.allclose(W, D, atol=1e-12) for D in distinct):
            distinct.append(W)
    assert len(distinct) == 3
    for W in Ws[1:-1]:
        np.testing.assert_allclose(W, Ws[1], atol=1e-12)


def test_sample_covariance_filter_woodbury():
    # push-through identity: R_OI (R_II + lam I)^-1 X = X_O G (G + lam I)^-1,
    # G = X^H X / M, an independent route through an M x M system
    rng = np.random.default_rng(3)
    M, Wn, B, off, lam = 40, 50, 30, 10, 0.01
    X = (rng.standard_normal((Wn, M)) + 1j * rng.standard_normal((Wn, M))) / np.sqrt(2)
    R = O.sample_covariance(X.T)
    np.testing.assert_allclose(R, X @ np.conj(X).T / M, atol=1e-13)
    assert np.linalg.matrix_rank(R) == M
    W = O.lmmse._filter(R[off:off + B], R, lam)
    Gm = np.conj(X).T @ X / M
    lhs = W @ X
    rhs = X[off:off + B] @ Gm @ np.linalg.inv(Gm + lam * np.eye(M))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9, atol=1e-11)


def test_apply_matches_brute_force_loops():
    sb = make_slot_batch(**TINY, slots=1)
    X = O.despread(sb.y, sb.pilots)
    R = _R_exp(72)
    for B, Wn in ((12, 12), (12, 24), (72, 72)):
        Ws, starts = O.block_filters(R, B, Wn, 0.05)
        out = O.apply_filters(Ws, starts, B, X)
        ref = np.zeros_like(out)
        for m in range(X.shape[1]):
            for k in range(X.shape[2]):
                for b, s in enumerate(starts):
                    for i in range(B):
                        acc = 0j
                        for j in range(Wn):
                            acc += Ws[b][i, j] * X[0, m, k, s + j]
                        ref[0, m, k, b * B + i] = acc
        np.testing.assert_allclose(out, ref, atol=1e-12)


# ------------------------------------------------------------------ error
def test_expected_mse_ls_and_full_closed_forms():
    R = _R_exp(72)
    lam = 0.05
    # LS = identity filter: error is exactly the LS noise lam
    Ws = [np.eye(12)] * 6
    assert abs(O.expected_mse(R, lam, Ws, list(range(0, 72, 12)), 12) - lam) < 1e-14
    # matched full LMMSE: tr(R - W R^H) / N (valid only at the optimum)
    W = O.full_lmmse_filter(R, lam)
    mse = O.expected_mse(R, lam, [W], [0], 72)
    assert abs(mse - np.trace(R - W @ np.conj(R).T).real / 72) < 1e-12


def test_monte_carlo_matches_closed_form_tiny():
    # NMSE of the oracle estimator over many seeded slots vs the closed form
    nslots = 40
    sb = make_slot_batch(**TINY, slots=nslots, config_id=0)
    R = _R_exp(72)
    lam = sb.sigma2 / 2
    for B, Wn in ((12, 12), (72, 72), (12, 36)):
        est = O.estimate(sb.y, sb.pilots, sb.sigma2, B, Wn, "exp", N_fft=128, tau=2.0, taps=8)
        mc = np.mean(np.abs(est - sb.H) ** 2)
        Ws, st = O.block_filters(R, B, Wn, lam)
        cf = O.expected_mse(R, lam, Ws, st, B)
        # relative Monte Carlo error of a mean of |e|^2 (correlated along n)
        assert abs(mc - cf) / cf < 0.06, (B, Wn, mc, cf)


def test_expected_nmse_ordering_and_independent_values():
    # Closed-form NMSE of the paper-sized system (tau 4, SNR 10 dB), compared
    # with values computed independently from the same formula when the
    # workloads were specified: LS -20.79, full -37.03, non-overlap B=100
    # -34.61, overlap 150/100 -36.13 dB (true R); uniform design overlap
    # -30.67 dB.
    N, K, sig2 = 1200, 12, 0.1
    lam = sig2 / K
    n = np.arange(N)
    R = O.toeplitz_from_r(lambda d: O.r_exponential(d, 4.0, 72, 2048), n, n)
    Ru = O.toeplitz_from_r(lambda d: O.r_uniform(d, 144, 2048), n, n)
    vals = {}
    vals["ls"] = 10 * np.log10(lam)
    W = O.full_lmmse_filter(R, lam)
    vals["full"] = 10 * np.log10(O.expected_mse(R, lam, [W], [0], N))
    Ws, st = O.block_filters(R, 100, 100, lam)
    vals["non"] = 10 * np.log10(O.expected_mse(R, lam, Ws, st, 100))
    Ws, st = O.block_filters(R, 100, 150, lam)
    vals["ovl"] = 10 * np.log10(O.expected_mse(R, lam, Ws, st, 100))
    Ws, st = O.block_filters(Ru, 100, 150, lam)
    vals["uni"] = 10 * np.log10(O.expected_mse(R, lam, Ws, st, 100))
    ref = dict(ls=-20.79, full=-37.03, non=-34.61, ovl=-36.13, uni=-30.67)
    for k, v in ref.items():
        assert abs(vals[k] - v) < 0.006, (k, vals[k], v)
    assert vals["ls"] > vals["uni"] > vals["non"] > vals["ovl"] > vals["full"]


def test_sample_estimate_full_rank_window_agrees_with_woodbury_route():
    sb = make_slot_batch(M=16, K=2, N=24, N_fft=64, taps=4, tau=2.0, snr_db=10.0, slots=1)
    est, hls = O.estimate(sb.y, sb.pilots, sb.sigma2, 8, 12, "sample", return_ls=True)
    lam = sb.sigma2 / 2
    starts, offs = O.window_starts(24, 8, 12)
    for k in range(2):
        for b, (s, off) in enumerate(zip(starts, offs)):
            X = hls[0, :, k, s:s + 12].T                # Wn x M
            Gm = np.conj(X).T @ X / 16
            ref = X[off:off + 8] @ Gm @ np.linalg.inv(Gm + lam * np.eye(16))
            np.testing.assert_allclose(est[0, :, k, b * 8:(b + 1) * 8], ref.T, rtol=1e-9, atol=1e-12)


def test_exponential_pdp_generator_matches_oracle_profile():
    np.testing.assert_allclose(exponential_pdp(4.0, 72), O.lmmse._exp_profile(4.0, 72), rtol=1e-15)
