"""Robustness sweeps of Fig. 7(b-d) on the GPU comb 12W estimator
(qualitative trends, as the text describes them, on seeded Table III-like
data: 16 antennas, 4 UEs, N=1200 of 2048):
  * assumed channel length L = 1..15 with a true 7-tap channel: the error is
    lowest near the true length, rises steeply below it and mildly above;
  * design SNR 0..40 dB with a true 25 dB: robust when the design SNR is at
    least the true one;
  * a 2-sample timing error (a linear phase over the subcarriers): a slight
    change only."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import CombPlan
from synth import make_comb_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _nmse(dev, cb, L, sigma2, y=None, H=None):
    y = cb.y if y is None else y
    H = cb.H if H is None else H
    with CombPlan(M=16, K=4, N=1200, N_fft=2048, comb=12, kind="12w", rsource="uniform", L=L,
                  sigma2=sigma2, max_slots=cb.y.shape[0]) as pl:
        out = pl.estimate(torch.from_numpy(np.ascontiguousarray(y)).to(dev),
                          torch.from_numpy(cb.pilots).to(dev)).cpu().numpy()
    return O.nmse_db(out, H)


def test_assumed_channel_length_sweep(dev):
    cb = make_comb_batch(M=16, K=4, N=1200, N_fft=2048, powers_db=[0] * 7, snr_db=25.0, slots=4)
    Ls = [1, 3, 5, 6, 7, 8, 9, 11, 15]
    e = {L: _nmse(dev, cb, float(L), cb.sigma2) for L in Ls}
    print("NMSE by assumed L:", {k: round(v, 2) for k, v in e.items()}, flush=True)
    assert min(e, key=e.get) in (6, 7, 8)
    assert e[1] - e[7] > 6.0          # steep below the true length
    assert e[15] - e[7] < 2.0         # mild above it


def test_design_snr_sweep(dev):
    cb = make_comb_batch(M=16, K=4, N=1200, N_fft=2048, powers_db=[-2, -8, -10, -12, -15, -18],
                         snr_db=25.0, slots=4)
    e = {sf: _nmse(dev, cb, 8.0, 10 ** (-sf / 10)) for sf in (0, 10, 20, 25, 30, 40)}
    print("NMSE by design SNR:", {k: round(v, 2) for k, v in e.items()}, flush=True)
    best = min(e.values())
    for sf in (25, 30, 40):
        assert e[sf] - best < 1.0
    assert e[0] - best > 6.0


def test_timing_error_changes_little(dev):
    cb = make_comb_batch(M=16, K=4, N=1200, N_fft=2048, powers_db=[-2, -5, -8, -10, -12, -15, -18],
                         snr_db=25.0, slots=4)
    ramp = np.exp(-2j * np.pi * 2 * np.arange(1200) / 2048)
    y2 = (cb.y * ramp[None, None, :]).astype(np.complex64)
    H2 = cb.H * ramp[None, None, None, :]
    e0 = _nmse(dev, cb, 7.0, cb.sigma2)
    e2 = _nmse(dev, cb, 7.0, cb.sigma2, y=y2, H=H2)
    print(f"NMSE without / with a 2-sample timing error: {e0:.2f} / {e2:.2f} dB", flush=True)
    assert abs(e2 - e0) < 2.0
