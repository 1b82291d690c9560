"""FP64 oracle of the comb-pilot estimators 3W-LMMSE and 12W-LMMSE (Sec. IV-B,
Tables I-II, the 3W weights and P, zero-order hold of Sec. IV-C).  Test
infrastructure only, like the rest of this package.

Pilot structure (Sec. II, eq. 6): a pilot OFDM symbol carries the pilot of
UE s (0-based here) on the comb tones s, s + S, s + 2S, ... (N/S tones), so
the received pilot symbol is y[slot][m][n] = H_{u(n)}[n] x[n] + w with u(n) =
n mod S; x[n] is the pilot on subcarrier n (that of its UE).

Readings:
  * P in the 3W weights is the inverse (R_II + sigma^2/sigma_s^2 I)^-1, as in
    eq. 13 / eq. 17 (the printed P lacks the inverse).
  * One unit-modulus pilot symbol per LS value: sigma_s^2 = 1, so the
    regulariser is lam = sigma2 itself.
  * Zero-order hold (3W): every subcarrier without an estimate takes the
    latest estimated subcarrier below it; subcarriers below the first
    estimate take the first one.
  * 3W outputs of a UE's last tone that fall past subcarrier N are dropped
    (the table is printed for UE 1 only, whose outputs all fit).
"""
from __future__ import annotations

import numpy as np

from .lmmse import C128, _filter, comb_group_table, toeplitz_from_r


def comb_ls(y: np.ndarray, pilots: np.ndarray) -> np.ndarray:
    """LS on every subcarrier of the pilot symbol, eq. 9: Y(k) / X(k).
    y: [S][M][N], pilots: [N].  Returns complex128 [S][M][N]."""
    return np.asarray(y).astype(C128) / np.asarray(pilots).astype(C128)[None, None, :]


def comb_groups(N: int, S: int, ue: int, kind: str):
    """The groups of UE `ue` (0-based) as 0-based (outputs, LS tones) lists,
    from the 1-based tables (Tables I and II).  3W outputs that fall past the
    band (UE offsets of S/3 and more on the last tone) are dropped."""
    rows = comb_group_table(N, S, ue + 1, kind)
    return [([o - 1 for o in outs if o <= N], [t - 1 for t in ls]) for (_, outs, _, ls) in rows]


def comb_filters(N: int, S: int, ue: int, kind: str, r_of_d, lam: float):
    """W_b = R_OI (R_II + lam I)^-1 of every group b of UE `ue`, with
    R[a, b] = r(a - b) over the subcarrier indices (eq. 13, eq. 17)."""
    out = []
    for outs, tones in comb_groups(N, S, ue, kind):
        R_oi = toeplitz_from_r(r_of_d, outs, tones)
        R_ii = toeplitz_from_r(r_of_d, tones, tones)
        out.append(_filter(R_oi, R_ii, lam))
    return out


def zero_order_hold(vals: np.ndarray, have: np.ndarray) -> np.ndarray:
    """Fill the subcarriers without an estimate (have[n] False) from the
    latest estimated one below, or from the first one below none."""
    vals = np.array(vals, dtype=C128)
    idx = np.flatnonzero(have)
    if idx.size == 0:
        raise ValueError("no estimate to hold")
    out = vals.copy()
    last = idx[0]
    for n in range(vals.shape[-1]):
        if have[n]:
            last = n
        out[..., n] = vals[..., last]
    return out


def comb_estimate(y, pilots, sigma2: float, S: int, ues, kind: str, r_of_d) -> np.ndarray:
    """3W / 12W estimate of the UEs `ues` (0-based comb offsets).
    y: [slots][M][N] pilot symbol, pilots: [N].  Returns [slots][M][len(ues)][N]."""
    ls = comb_ls(y, pilots)
    nsl, M, N = ls.shape
    out = np.zeros((nsl, M, len(ues), N), dtype=C128)
    for ui, ue in enumerate(ues):
        Ws = comb_filters(N, S, ue, kind, r_of_d, sigma2)
        have = np.zeros(N, dtype=bool)
        est = np.zeros((nsl, M, N), dtype=C128)
        for W, (outs, tones) in zip(Ws, comb_groups(N, S, ue, kind)):
            est[:, :, outs] = ls[:, :, tones] @ W.T
            have[outs] = True
        out[:, :, ui, :] = est if have.all() else zero_order_hold(est, have)
    return out


def comb_ls_hold(y, pilots, S: int, ues) -> np.ndarray:
    """The LS values on each UE's tones held over the subcarriers between
    them (the zero-order-hold LS baseline of Sec. IV-C)."""
    ls = comb_ls(y, pilots)
    nsl, M, N = ls.shape
    out = np.zeros((nsl, M, len(ues), N), dtype=C128)
    for ui, ue in enumerate(ues):
        have = np.zeros(N, dtype=bool)
        have[ue::S] = True
        est = np.where(have[None, None, :], ls, 0)
        out[:, :, ui, :] = zero_order_hold(est, have)
    return out


def comb_ls_linear(y, pilots, S: int, ues, fold: int | None = None) -> np.ndarray:
    """Interpolated-LS baselines (Sec. IV-A-1, interpolated LS; comparison lines of Sec. V).

    fold=None: each subcarrier linearly interpolates the LS values of the two
    UE tones around it (the nearest tone's value outside the first..last
    tone).  fold=3 ("3-fold interpolated LS"): the same linear interpolation
    evaluated only at the 3W output positions tone + j S/3, then the
    zero-order hold of the 3W estimator fills the rest."""
    ls = comb_ls(y, pilots)
    nsl, M, N = ls.shape
    out = np.zeros((nsl, M, len(ues), N), dtype=C128)
    for ui, ue in enumerate(ues):
        tones = np.arange(ue, N, S)
        vals = ls[:, :, tones]
        def lin(p):
            p = np.asarray(p, dtype=np.float64)
            res = np.empty((nsl, M) + p.shape, dtype=C128)
            for idx, q in np.ndenumerate(p):
                if q <= tones[0]:
                    res[(slice(None), slice(None)) + idx] = vals[:, :, 0]
                elif q >= tones[-1]:
                    res[(slice(None), slice(None)) + idx] = vals[:, :, -1]
                else:
                    i = int((q - ue) // S)
                    f = (q - tones[i]) / S
                    res[(slice(None), slice(None)) + idx] = (1 - f) * vals[:, :, i] + f * vals[:, :, i + 1]
            return res
        if fold is None:
            out[:, :, ui, :] = lin(np.arange(N))
        else:
            have = np.zeros(N, dtype=bool)
            est = np.zeros((nsl, M, N), dtype=C128)
            for t in tones:
                for j in range(fold):
                    q = t + j * (S // fold)
                    if q < N:
                        est[:, :, q] = lin(np.array([q]))[:, :, 0]
                        have[q] = True
            out[:, :, ui, :] = zero_order_hold(est, have)
    return out


def comb_ls_quadratic(y, pilots, S: int, ues) -> np.ndarray:
    """Second-order polynomial interpolated LS (Sec. IV-A-1, the interpolated LS
    estimators).  Reading: a subcarrier between a UE's tones i and i+1 takes
    the quadratic through the LS values of tones i-1, i, i+1 (tones 0, 1, 2
    in the first interval); outside the first..last tone the nearest tone's
    value is held, as for the linear form."""
    ls = comb_ls(y, pilots)
    nsl, M, N = ls.shape
    out = np.zeros((nsl, M, len(ues), N), dtype=C128)
    for ui, ue in enumerate(ues):
        tones = np.arange(ue, N, S)
        vals = ls[:, :, tones]
        nt = len(tones)
        for p in range(N):
            if p <= tones[0]:
                out[:, :, ui, p] = vals[:, :, 0]
            elif p >= tones[-1]:
                out[:, :, ui, p] = vals[:, :, -1]
            else:
                i = (p - ue) // S
                m = min(max(i - 1, 0), nt - 3)
                x = (p - ue) / S                 # position in tone units
                nodes = [m, m + 1, m + 2]
                for a in nodes:                  # Lagrange basis through the three tones
                    wa = 1.0
                    for b in nodes:
                        if b != a:
                            wa *= (x - b) / (a - b)
                    out[:, :, ui, p] += wa * vals[:, :, a]
    return out


def natural_spline_second_derivatives(v: np.ndarray) -> np.ndarray:
    """Second derivatives (per unit knot spacing) of the natural cubic spline
    through equally spaced values v[..., 0..n-1]: zero at both ends, and on
    the interior knots the continuity of the first derivative,
    M[i-1] + 4 M[i] + M[i+1] = 6 (v[i-1] - 2 v[i] + v[i+1])."""
    n = v.shape[-1]
    Mdd = np.zeros(v.shape, dtype=C128)
    if n <= 2:
        return Mdd
    T = 4.0 * np.eye(n - 2) + np.eye(n - 2, k=1) + np.eye(n - 2, k=-1)
    rhs = 6.0 * (v[..., :-2] - 2.0 * v[..., 1:-1] + v[..., 2:])
    Mdd[..., 1:-1] = np.linalg.solve(T, rhs.reshape(-1, n - 2).T).T.reshape(rhs.shape)
    return Mdd


def comb_ls_spline(y, pilots, S: int, ues) -> np.ndarray:
    """Cubic-spline interpolated LS (Sec. IV-A-1, the interpolated LS estimators).
    Reading: the natural cubic spline (zero second derivative at the first
    and last tone) through the LS values of a UE's tones, real and imaginary
    parts alike; outside the first..last tone the nearest tone's value is
    held.  On the interval between tones i and i+1, with u the fraction of
    the way, the spline is (1-u) v_i + u v_{i+1} + ((1-u)^3 - (1-u)) M_i / 6
    + (u^3 - u) M_{i+1} / 6."""
    ls = comb_ls(y, pilots)
    nsl, M, N = ls.shape
    out = np.zeros((nsl, M, len(ues), N), dtype=C128)
    for ui, ue in enumerate(ues):
        tones = np.arange(ue, N, S)
        vals = ls[:, :, tones]
        Mdd = natural_spline_second_derivatives(vals)
        for p in range(N):
            if p <= tones[0]:
                out[:, :, ui, p] = vals[:, :, 0]
            elif p >= tones[-1]:
                out[:, :, ui, p] = vals[:, :, -1]
            else:
                i = (p - ue) // S
                u = (p - tones[i]) / S
                out[:, :, ui, p] = ((1 - u) * vals[:, :, i] + u * vals[:, :, i + 1]
                                    + ((1 - u) ** 3 - (1 - u)) * Mdd[:, :, i] / 6
                                    + (u ** 3 - u) * Mdd[:, :, i + 1] / 6)
    return out
