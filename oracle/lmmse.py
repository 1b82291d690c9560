"""FP64 oracle of the forward path (test infrastructure only; see package doc).

Notation: M BS antennas, K users, N used subcarriers (bins 0..N-1 of an
N_fft-point FFT), block size B, window Wn.  Arrays are [S][M][K][N] with the
subcarrier axis last.  Every routine works in complex128.

Readings of points the paper leaves open (each one is applied below):
  * LS noise: K pilot symbols with a unit-modulus K x K DFT cover code give an
    LS estimate whose noise variance is lam = sigma2 / K; the filters use lam
    where eq. 13 / eq. 17 write sigma^2 / sigma_s^2.
  * eq. 16 / r_d: the "N" in the exponent is the FFT size N_fft (the channel
    length L is in samples, the subcarrier spacing is 1/N_fft).
  * "Exponential" fixed design: the discrete tap sum with the generator's
    profile; the uniform profile of eq. 16 is its tau -> infinity limit.
  * Band edges: windows are shifted inside the band, never truncated
    (Tables I-II); start_b = clamp(b*B - floor((Wn-B)/2), 0, N - Wn).
  * Sample covariance: raw (1/M) sum over antennas of h h^H per (slot, user,
    window), no mean removal and no noise debiasing.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

C128 = np.complex128


# --------------------------------------------------------------------------
# Pilots and LS (Sec. IV-A-1, eq. 8-9; Sec. IV-C "channel_estimation.c")
# --------------------------------------------------------------------------
def cover_code(K: int) -> np.ndarray:
    """c[k, t] = exp(-j 2 pi k t / K): user k's cover over pilot symbols t."""
    c = np.empty((K, K), dtype=C128)
    for k in range(K):
        for t in range(K):
            c[k, t] = np.exp(-2j * np.pi * k * t / K)
    return c


def despread(y: np.ndarray, pilots: np.ndarray) -> np.ndarray:
    """LS estimate per (antenna, user, subcarrier).

    eq. 9 gives H_LS = Y(k) / X_s(k) for one pilot symbol.  With K code-spread
    pilot symbols, user k's received pilot is first isolated by correlating
    with its cover, z_k = (1/K) sum_t conj(c[k,t]) y_t, and then divided by
    the pilot symbol x_k[n] (eq. 9).
    y: [S][M][K(t)][N]; pilots: [K][N].  Returns [S][M][K][N] complex128.
    """
    y = np.asarray(y).astype(C128)
    K = y.shape[2]
    c = cover_code(K)
    z = np.einsum("kt,smtn->smkn", np.conj(c), y) / K
    return z / np.asarray(pilots).astype(C128)[None, None, :, :]


# --------------------------------------------------------------------------
# Subcarrier correlation (Sec. IV-A-2, eq. 14-16 and r_d)
# --------------------------------------------------------------------------
def r_uniform(d, L: float, N_fft: int) -> np.ndarray:
    """r_d of the fixed design (eq. 16 written as a function of d = ka - kb):
    1 at d = 0, else (1 - exp(-j 2 pi L d / N_fft)) / (j 2 pi L d / N_fft)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.ones(d.shape, dtype=C128)
    nz = d != 0
    a = 2j * np.pi * float(L) * d[nz] / float(N_fft)
    out[nz] = (1.0 - np.exp(-a)) / a
    return out


def _exp_profile(tau: float, taps: int) -> np.ndarray:
    l = np.arange(int(taps), dtype=np.float64)
    w = np.exp(-l / float(tau))
    return w / w.sum()


def r_exponential(d, tau: float, taps: int, N_fft: int) -> np.ndarray:
    """E{H(a) H(b)^*} for zero-mean taps at integer delays l < taps with powers
    p_l proportional to exp(-l / tau) (the profile of Sec. IV-A), d = a - b:
    r_d = sum_l p_l exp(-j 2 pi l d / N_fft)."""
    d = np.asarray(d, dtype=np.float64)
    p = _exp_profile(tau, taps)
    l = np.arange(int(taps), dtype=np.float64)
    ph = np.exp(-2j * np.pi * np.multiply.outer(d, l) / float(N_fft))
    return (ph * p).sum(axis=-1)


def r_exponential_cont(d, tau: float, L: float, N_fft: int) -> np.ndarray:
    """Continuous-delay exponential profile on [0, L) (cross-check only):
    r_d = (1 - e^{-L q}) / (tau (1 - e^{-L/tau}) q),  q = 1/tau + j 2 pi d / N_fft.
    It tends to the uniform r_d as tau -> infinity."""
    d = np.asarray(d, dtype=np.float64)
    q = 1.0 / float(tau) + 2j * np.pi * d / float(N_fft)
    return (1.0 - np.exp(-float(L) * q)) / (float(tau) * (1.0 - np.exp(-float(L) / float(tau))) * q)


def toeplitz_from_r(r_of_d, rows, cols) -> np.ndarray:
    """R[a, b] = r(rows[a] - cols[b]) (the correlation depends only on the
    subcarrier difference, Sec. IV-A-2)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    d = rows[:, None] - cols[None, :]
    # r is evaluated once per distinct difference (the same values as
    # evaluating it entry by entry)
    d0 = int(d.min()) if d.size else 0
    vals = np.asarray(r_of_d(np.arange(d0, int(d.max()) + 1 if d.size else 0)), dtype=C128)
    return vals[d - d0]


def sample_covariance(x: np.ndarray) -> np.ndarray:
    """Raw sample covariance over antennas: x is [M][W] (one user, one window,
    every antenna); returns (1/M) sum_m x_m x_m^H, [W][W]."""
    x = np.asarray(x).astype(C128)
    M = x.shape[0]
    R = np.zeros((x.shape[1], x.shape[1]), dtype=C128)
    for m in range(M):
        R += np.outer(x[m], np.conj(x[m]))
    return R / M


# --------------------------------------------------------------------------
# Block plan (Sec. IV-B; Tables I-II)
# --------------------------------------------------------------------------
def window_starts(n_units: int, out_per_block: int, win: int):
    """Window start of every output block.

    Output block b covers units [b*B, (b+1)*B); its input window of `win`
    units is centred on it and shifted (not truncated) to stay inside the
    band: start_b = clamp(b*B - floor((win - B)/2), 0, n_units - win).
    Returns (starts, offsets) with offsets_b = b*B - start_b.
    """
    B = int(out_per_block)
    if n_units % B != 0:
        raise ValueError("n_units must be a multiple of the block size")
    if not (B <= win <= n_units):
        raise ValueError("need B <= win <= n_units")
    halo = (win - B) // 2
    starts, offs = [], []
    for b in range(n_units // B):
        s = min(max(b * B - halo, 0), n_units - win)
        starts.append(s)
        offs.append(b * B - s)
    return starts, offs


def comb_group_table(N: int, S: int, ue: int, kind: str):
    """Group table of the comb-pilot 3W / 12W estimators (Tables I and II).

    UE `ue` (1-based) owns pilot tones ue, ue+S, ue+2S, ... (1-based
    subcarriers, N/S tones).  Rows are (index, output subcarriers, filter id,
    LS subcarriers), all 1-based.  3W: output group b holds tone b and the two
    subcarriers S/3 and 2S/3 above it, window = 3 tones.  12W: output group b
    holds subcarriers 12b+1..12b+12, window = 12 tones.  Filter ids number the
    distinct output-vs-window placements in order of first use.
    """
    n_tones = N // S
    tones = [ue + i * S for i in range(n_tones)]
    if kind == "3w":
        win, outs = 3, [[tones[b] + j * (S // 3) for j in range(3)] for b in range(n_tones)]
    elif kind == "12w":
        win, outs = 12, [[S * b + 1 + j for j in range(S)] for b in range(n_tones)]
    else:
        raise ValueError(kind)
    starts, _ = window_starts(n_tones, 1, win)
    rows, ids = [], {}
    for b in range(n_tones):
        ls = tones[starts[b]: starts[b] + win]
        key = tuple(o - ls[0] for o in outs[b])
        if key not in ids:
            ids[key] = len(ids) + 1
        rows.append((b + 1, outs[b], ids[key], ls))
    return rows


# --------------------------------------------------------------------------
# Filters (eq. 13 / eq. 17, partitioned per Sec. IV-B)
# --------------------------------------------------------------------------
def _filter(R_oi: np.ndarray, R_ii: np.ndarray, lam: float) -> np.ndarray:
    """W = R_OI (R_II + lam I)^-1 via a Cholesky solve of the Hermitian system."""
    A = R_ii + float(lam) * np.eye(R_ii.shape[0])
    cf = sla.cho_factor(A, lower=True)
    return np.conj(sla.cho_solve(cf, np.conj(R_oi).T)).T


def block_filters(R: np.ndarray, B: int, Wn: int, lam: float):
    """Partitioned filters from an N x N correlation R (eq. 13 restricted to
    each block): W_b = R[O_b, I_b] (R[I_b, I_b] + lam I)^-1.
    Returns (list of B x Wn filters, window starts)."""
    N = R.shape[0]
    starts, _ = window_starts(N, B, Wn)
    Ws = []
    for b, s in enumerate(starts):
        I = np.arange(s, s + Wn)
        O = np.arange(b * B, (b + 1) * B)
        Ws.append(_filter(R[np.ix_(O, I)], R[np.ix_(I, I)], lam))
    return Ws, starts


def full_lmmse_filter(R: np.ndarray, lam: float) -> np.ndarray:
    """Full-band LMMSE weight (eq. 13): W = R (R + lam I)^-1, N x N."""
    return _filter(R, R, lam)


def apply_filters(Ws, starts, B: int, X: np.ndarray) -> np.ndarray:
    """eq. 12 per block: Hhat[..., O_b] = W_b H_LS[..., I_b] for every column."""
    X = np.asarray(X).astype(C128)
    out = np.zeros_like(X)
    for b, (W, s) in enumerate(zip(Ws, starts)):
        Wn = W.shape[1]
        out[..., b * B:(b + 1) * B] = X[..., s:s + Wn] @ W.T
    return out


def estimate(y, pilots, sigma2: float, B: int, Wn: int, rsource: str,
             N_fft: int | None = None, L: float | None = None,
             tau: float | None = None, taps: int | None = None,
             R: np.ndarray | None = None, return_ls: bool = False):
    """End-to-end oracle: despread -> R -> block filters -> apply.

    rsource: 'uniform' (eq. 16 with L), 'exp' (discrete profile tau, taps),
    'user' (caller's N x N R) or 'sample' (per slot and user sample covariance
    over the antennas, separately in every window).
    """
    H_ls = despread(y, pilots)
    S, M, K, N = H_ls.shape
    lam = float(sigma2) / K
    n = np.arange(N)
    if rsource in ("uniform", "exp", "user"):
        if rsource == "uniform":
            R = toeplitz_from_r(lambda d: r_uniform(d, L, N_fft), n, n)
        elif rsource == "exp":
            R = toeplitz_from_r(lambda d: r_exponential(d, tau, taps, N_fft), n, n)
        Ws, starts = block_filters(R, B, Wn, lam)
        out = apply_filters(Ws, starts, B, H_ls)
    elif rsource == "sample":
        out = np.zeros_like(H_ls)
        starts, offs = window_starts(N, B, Wn)
        for s in range(S):
            for k in range(K):
                for b, (st, off) in enumerate(zip(starts, offs)):
                    X = H_ls[s, :, k, st:st + Wn]            # [M][Wn]
                    Rw = sample_covariance(X)
                    W = _filter(Rw[off:off + B, :], Rw, lam)
                    out[s, :, k, b * B:(b + 1) * B] = X @ W.T
    else:
        raise ValueError(rsource)
    return (out, H_ls) if return_ls else out


# --------------------------------------------------------------------------
# Expected error and metrics
# --------------------------------------------------------------------------
def expected_mse(R_true: np.ndarray, lam_true: float, Ws, starts, B: int) -> float:
    """Expected squared error per coefficient of the block estimator with
    filters Ws when the channel has correlation R_true and the LS noise is
    white with variance lam_true:
      (1/N) sum_b tr(R_OO - W R_IO - R_OI W^H + W (R_II + lam I) W^H)."""
    N = R_true.shape[0]
    tot = 0.0
    for b, (W, s) in enumerate(zip(Ws, starts)):
        Wn = W.shape[1]
        I = np.arange(s, s + Wn)
        O = np.arange(b * B, (b + 1) * B)
        Roo = R_true[np.ix_(O, O)]
        Roi = R_true[np.ix_(O, I)]
        Rio = R_true[np.ix_(I, O)]
        Aii = R_true[np.ix_(I, I)] + lam_true * np.eye(Wn)
        t = np.trace(Roo - W @ Rio - Roi @ np.conj(W).T + W @ Aii @ np.conj(W).T)
        tot += t.real
    return tot / N


def nmse(est, truth) -> float:
    """sum |est - truth|^2 / sum |truth|^2 over the whole batch."""
    est = np.asarray(est).astype(C128)
    truth = np.asarray(truth).astype(C128)
    return float(np.sum(np.abs(est - truth) ** 2) / np.sum(np.abs(truth) ** 2))


def nmse_db(est, truth) -> float:
    return 10.0 * np.log10(nmse(est, truth))


def discrepancy_db(est, ref) -> float:
    """10 log10(||est - ref||^2 / ||ref||^2)."""
    return nmse_db(est, ref)
