"""Seeded generator of uplink pilot slots.

Channel model (Sec. II, eq. 1-5, with the power-delay profile of Sec. IV-A):
each (slot s, BS antenna m, user k) link is an integer-delay multipath channel
with taps h_l ~ CN(0, p_l), l = 0..L_taps-1, where p_l is an exponential
profile with decay tau_rms (in samples) normalised to sum 1.  With a cyclic
prefix at least as long as the channel, the per-subcarrier model of eq. 5
holds exactly, so the generator works in the frequency domain:

    H[s,m,k,n] = sum_l h_l exp(-j 2 pi l n / N_fft),   n = 0..N-1

(the used subcarriers are the contiguous bins 0..N-1).

Pilots: user k sends a unit-modulus QPSK sequence x_k[n] on every used
subcarrier of K pilot OFDM symbols t = 0..K-1, multiplied by the cover code
c[k,t] = exp(-j 2 pi k t / K) (one row of a K x K DFT).  Antenna m receives

    y[s,m,t,n] = sum_k c[k,t] x_k[n] H[s,m,k,n] + w[s,m,t,n],
    w ~ CN(0, sigma2),  sigma2 = 10^(-SNR/10).

Layouts: y and H are [S][M][K][N] (t or k third), contiguous in n.

Seeds: numpy PCG64 streams; pilots from PILOT_SEED, slot s of config c from
slot_seed(c, s).  Nothing here implements the estimator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PILOT_SEED = 180205427


def slot_seed(config_id: int, slot: int, base: int = PILOT_SEED) -> int:
    """Seed of one slot: base + 1000 * config + slot."""
    return int(base + 1000 * int(config_id) + int(slot))


# Workload shapes.  "taps" is the number of integer-delay taps the generator
# draws; B / Wn are the partition sizes exercised on that shape.
CONFIGS = {
    "tiny": dict(config_id=0, M=8, K=2, N_fft=128, N=72, taps=8, tau=2.0,
                 snr_db=10.0, B=12, Wn=12, slots=1),
    "paper": dict(config_id=1, M=128, K=12, N_fft=2048, N=1200, taps=72,
                  tau=4.0, snr_db=10.0, B=100, Wn=150, slots=1),
    "precision": dict(config_id=2, M=128, K=12, N_fft=2048, N=1200, taps=72,
                      tau=4.0, snr_db=10.0, B=100, Wn=150, slots=64),
    "diff": dict(config_id=3, M=128, K=12, N_fft=2048, N=1200, taps=72,
                 tau=(2.0, 24.0), snr_db=10.0, B=100, Wn=150, slots=16),
    "large": dict(config_id=4, M=256, K=24, N_fft=4096, N=3300, taps=144,
                  tau=32.0, snr_db=15.0, B=132, Wn=198, slots=32),
}


def exponential_pdp(tau_rms: float, taps: int) -> np.ndarray:
    """Tap powers p_l proportional to exp(-l / tau_rms), l < taps, sum 1."""
    l = np.arange(int(taps), dtype=np.float64)
    w = np.exp(-l / float(tau_rms))
    return w / w.sum()


def make_pilots(K: int, N: int, seed: int = PILOT_SEED) -> np.ndarray:
    """Unit-modulus QPSK pilots x_k[n] = ((+-1) + j(+-1))/sqrt(2), [K][N] c64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=(K, N, 2))
    sym = ((1 - 2 * bits[..., 0]) + 1j * (1 - 2 * bits[..., 1])) / np.sqrt(2.0)
    return sym.astype(np.complex64)


@dataclass
class SlotBatch:
    y: np.ndarray            # [S][M][K][N] complex64, received pilot symbols
    pilots: np.ndarray       # [K][N] complex64
    sigma2: float            # receive noise variance per resource element
    H: np.ndarray | None     # [S][M][K][N] complex128 truth, or None
    tau: np.ndarray          # [S][K] tau_rms used per (slot, user)
    meta: dict = field(default_factory=dict)


def _draw_slot(rng, M, K, N, N_fft, taps, tau_k, sigma2, pilots, noiseless):
    """One slot: returns (y c64 [M][K][N], H c128 [M][K][N])."""
    h = np.empty((M, K, taps), dtype=np.complex128)
    g = rng.standard_normal((M, K, taps, 2))
    for k in range(K):
        p = exponential_pdp(tau_k[k], taps)
        h[:, k, :] = (g[:, k, :, 0] + 1j * g[:, k, :, 1]) * np.sqrt(p / 2.0)
    H = np.fft.fft(h, n=N_fft, axis=-1)[..., :N]
    v = H * pilots.astype(np.complex128)[None, :, :]
    # transmitted superposition over users with the DFT cover code:
    # y_t = sum_k exp(-j 2 pi k t / K) v_k  is a length-K DFT along k.
    y = np.fft.fft(v, axis=1)
    if not noiseless:
        w = rng.standard_normal((M, K, N, 2))
        y = y + (w[..., 0] + 1j * w[..., 1]) * np.sqrt(sigma2 / 2.0)
    return y.astype(np.complex64), H


def make_slot_batch(M: int, K: int, N: int, N_fft: int, taps: int, tau,
                    snr_db: float | None, slots: int = 1, config_id: int = 0,
                    first_slot: int = 0, want_truth: bool = True,
                    noiseless: bool = False, seed_base: int = PILOT_SEED,
                    pilot_seed: int = PILOT_SEED) -> SlotBatch:
    """Draw `slots` slots.

    tau: a scalar tau_rms for every (slot, user), or a (lo, hi) tuple from
    which tau_rms ~ U[lo, hi] is drawn per (slot, user).
    snr_db: per-user SNR 1/sigma2 in dB (ignored when noiseless).
    """
    if taps > N_fft:
        raise ValueError("taps must not exceed N_fft")
    pilots = make_pilots(K, N, pilot_seed)
    sigma2 = 0.0 if (noiseless or snr_db is None) else float(10.0 ** (-snr_db / 10.0))
    y = np.empty((slots, M, K, N), dtype=np.complex64)
    H = np.empty((slots, M, K, N), dtype=np.complex128) if want_truth else None
    taus = np.empty((slots, K), dtype=np.float64)
    for i in range(slots):
        rng = np.random.Generator(np.random.PCG64(slot_seed(config_id, first_slot + i, seed_base)))
        if isinstance(tau, (tuple, list)):
            tk = rng.uniform(float(tau[0]), float(tau[1]), size=K)
        else:
            tk = np.full(K, float(tau))
        taus[i] = tk
        yi, Hi = _draw_slot(rng, M, K, N, N_fft, taps, tk, sigma2, pilots, noiseless)
        y[i] = yi
        if want_truth:
            H[i] = Hi
    meta = dict(M=M, K=K, N=N, N_fft=N_fft, taps=taps, snr_db=snr_db,
                config_id=config_id, first_slot=first_slot)
    return SlotBatch(y=y, pilots=pilots, sigma2=sigma2, H=H, tau=taus, meta=meta)


def make_config_batch(name: str, slots: int | None = None, **over) -> SlotBatch:
    """Convenience: draw a batch with a named workload shape."""
    c = dict(CONFIGS[name])
    c.update(over)
    return make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"],
                           taps=c["taps"], tau=c["tau"], snr_db=c["snr_db"],
                           slots=slots if slots is not None else c["slots"],
                           config_id=c["config_id"],
                           first_slot=c.get("first_slot", 0),
                           want_truth=c.get("want_truth", True),
                           noiseless=c.get("noiseless", False))


@dataclass
class CombBatch:
    y: np.ndarray            # [S][M][N] complex64, the received comb pilot symbol
    pilots: np.ndarray       # [N] complex64, pilot of the UE owning each subcarrier
    sigma2: float
    H: np.ndarray            # [S][M][K][N] complex128 truth of the active UEs
    meta: dict = field(default_factory=dict)


def make_comb_batch(M: int, K: int, N: int, N_fft: int, powers_db, snr_db: float | None,
                    slots: int = 1, comb: int = 12, config_id: int = 5,
                    seed_base: int = PILOT_SEED, pilot_seed: int = PILOT_SEED) -> CombBatch:
    """Comb pilots (Sec. II, eq. 6): UE k < K owns the subcarriers k, k + comb,
    k + 2 comb, ... of one pilot OFDM symbol and sends a unit-modulus QPSK
    pilot there; subcarriers of inactive comb offsets carry noise only.
    Channel taps at integer delays 0..len(powers_db)-1 with the given powers
    in dB (normalised to sum 1), CN per (slot, antenna, UE)."""
    p = 10.0 ** (np.asarray(powers_db, dtype=np.float64) / 10.0)
    p = p / p.sum()
    taps = p.size
    rng0 = np.random.Generator(np.random.PCG64(pilot_seed + 7))
    bits = rng0.integers(0, 2, size=(N, 2))
    pil = (((1 - 2 * bits[:, 0]) + 1j * (1 - 2 * bits[:, 1])) / np.sqrt(2.0)).astype(np.complex64)
    sigma2 = 0.0 if snr_db is None else float(10.0 ** (-snr_db / 10.0))
    y = np.empty((slots, M, N), dtype=np.complex64)
    H = np.empty((slots, M, K, N), dtype=np.complex128)
    owner = np.arange(N) % comb
    for i in range(slots):
        rng = np.random.Generator(np.random.PCG64(slot_seed(config_id, i, seed_base)))
        g = rng.standard_normal((M, K, taps, 2))
        h = (g[..., 0] + 1j * g[..., 1]) * np.sqrt(p / 2.0)
        Hi = np.fft.fft(h, n=N_fft, axis=-1)[..., :N]
        H[i] = Hi
        yi = np.zeros((M, N), dtype=np.complex128)
        for k in range(K):
            sel = owner == k
            yi[:, sel] = Hi[:, k, sel] * pil[sel].astype(np.complex128)
        if sigma2 > 0:
            w = rng.standard_normal((M, N, 2))
            yi = yi + (w[..., 0] + 1j * w[..., 1]) * np.sqrt(sigma2 / 2.0)
        y[i] = yi.astype(np.complex64)
    meta = dict(M=M, K=K, N=N, N_fft=N_fft, comb=comb, powers_db=list(powers_db), snr_db=snr_db)
    return CombBatch(y=y, pilots=pil, sigma2=sigma2, H=H, meta=meta)


def make_data_symbols(H: np.ndarray, T: int, snr_db: float | None, seed: int = PILOT_SEED + 99):
    """Data OFDM symbols for detection (eq. 7 per subcarrier): unit-power
    QPSK X[s][t][k][n] from every user, received as Y[s][m][t][n] =
    sum_k H[s][m][k][n] X[s][t][k][n] + w, w ~ CN(0, sigma2).
    Returns (Y complex64, X complex128, sigma2)."""
    S, M, K, N = H.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=(S, T, K, N, 2))
    X = ((1 - 2 * bits[..., 0]) + 1j * (1 - 2 * bits[..., 1])) / np.sqrt(2.0)
    Y = np.einsum("smkn,stkn->smtn", H, X)
    sigma2 = 0.0 if snr_db is None else float(10.0 ** (-snr_db / 10.0))
    if sigma2 > 0:
        w = rng.standard_normal((S, M, T, N, 2))
        Y = Y + (w[..., 0] + 1j * w[..., 1]) * np.sqrt(sigma2 / 2.0)
    return Y.astype(np.complex64), X, sigma2
