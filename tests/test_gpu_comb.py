"""GPU parity of the comb-pilot 3W / 12W estimators (Sec. IV-B, Tables
I-II) against the FP64 oracle: the filter classes (FP64 design on the
device) and the whole estimate (LS on the comb tones, per-group filters,
zero-order hold) on seeded comb pilot symbols."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import CombPlan
from synth import make_comb_batch

pytestmark = pytest.mark.gpu

PROFILE = [-2, -8, -10, -12, -15, -18]   # 6 taps at delays 0..5 (dB)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _rd(c):
    if c.get("rsource", "uniform") == "uniform":
        return lambda d: O.r_uniform(d, c["L"], c["N_fft"])
    return lambda d: O.r_exponential(d, c["tau"], c["taps"], c["N_fft"])


def _plan(c, kind, sigma2):
    kw = dict(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], comb=c.get("comb", 12), kind=kind,
              sigma2=sigma2, max_slots=c["slots"])
    if c.get("rsource", "uniform") == "uniform":
        kw.update(rsource="uniform", L=c["L"])
    else:
        kw.update(rsource="exp", tau_rms=c["tau"], taps=c["taps"])
    return CombPlan(**kw)


CASES = [
    dict(M=4, K=3, N=240, N_fft=256, L=6.0, slots=2, snr=15.0),
    dict(M=16, K=4, N=1200, N_fft=2048, L=8.0, slots=2, snr=20.0),          # Table III-like system
    dict(M=3, K=12, N=600, N_fft=1024, L=8.0, slots=1, snr=10.0),           # every comb offset
    dict(M=2, K=4, N=1200, N_fft=2048, rsource="exp", tau=2.0, taps=6, slots=1, snr=20.0),
    dict(M=2, K=2, N=3300, N_fft=4096, L=16.0, slots=1, snr=20.0),          # 275 groups per UE
    dict(M=5, K=6, N=360, N_fft=512, L=6.0, comb=6, slots=1, snr=10.0),     # comb 6: 12W outputs 6
]


ODD_12W = [
    # odd spacing and odd N: neighbouring subcarriers in different groups, odd row length
    dict(M=2, K=3, N=255, N_fft=256, L=6.0, comb=5, slots=2, snr=15.0),
    dict(M=3, K=7, N=637, N_fft=1024, L=8.0, comb=7, slots=1, snr=20.0),
    # the largest filter set (S = 16) beside 768 tones: 7 columns staged, then 1
    dict(M=8, K=2, N=12288, N_fft=16384, L=8.0, comb=16, slots=1, snr=20.0),
]


@pytest.mark.parametrize("kind,c", [(k, c) for c in CASES for k in ("3w", "12w")]
                         + [("12w", c) for c in ODD_12W])
def test_comb_filters_and_estimate_match_oracle(dev, c, kind):
    print(f"comb {kind} {c}", flush=True)
    S = c.get("comb", 12)
    cb = make_comb_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], powers_db=PROFILE,
                         snr_db=c["snr"], slots=c["slots"], comb=S)
    rd = _rd(c)
    with _plan(c, kind, cb.sigma2) as pl:
        w = pl.get_filters().cpu().numpy()
        out = pl.estimate(_t(cb.y, dev), _t(cb.pilots, dev)).cpu().numpy()
    win = 3 if kind == "3w" else 12
    for k in range(c["K"]):
        Wo = O.comb_filters(c["N"], S, k, kind, rd, cb.sigma2)
        groups = O.comb_groups(c["N"], S, k, kind)
        nt = c["N"] // S
        for b, (outs, tones) in enumerate(groups):
            wst = min(max(b - (win - 1) // 2, 0), nt - win)
            assert tones[0] == k + S * wst
            Wg = w[k, b - wst, :len(outs), :]
            err = np.abs(Wg - Wo[b]).max() / np.abs(Wo[b]).max()
            assert err < 1e-10, (k, b, err)
    ref = O.comb_estimate(cb.y, cb.pilots, cb.sigma2, S, range(c["K"]), kind, rd)
    disc = O.discrepancy_db(out, ref)
    gap = abs(O.nmse_db(out, cb.H) - O.nmse_db(ref, cb.H))
    print(f"  discrepancy {disc:.1f} dB, NMSE gap {gap:.2e} dB", flush=True)
    assert disc < -120.0
    assert gap < 1e-4


@pytest.mark.parametrize("kind", ["ls_hold", "ls_linear", "ls_linear3"])
@pytest.mark.parametrize("c", [CASES[0], CASES[1], CASES[2], CASES[5]])
def test_interpolated_ls_baselines_match_oracle(dev, c, kind):
    print(f"comb {kind} {c}", flush=True)
    S = c.get("comb", 12)
    cb = make_comb_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], powers_db=PROFILE,
                         snr_db=c["snr"], slots=c["slots"], comb=S)
    with _plan(c, kind, cb.sigma2) as pl:
        out = pl.estimate(_t(cb.y, dev), _t(cb.pilots, dev)).cpu().numpy()
    if kind == "ls_hold":
        ref = O.comb_ls_hold(cb.y, cb.pilots, S, range(c["K"]))
    else:
        ref = O.comb_ls_linear(cb.y, cb.pilots, S, range(c["K"]), fold=3 if kind == "ls_linear3" else None)
    disc = O.discrepancy_db(out, ref)
    print(f"  discrepancy {disc:.1f} dB", flush=True)
    assert disc < -120.0


EDGE_LS = [
    dict(M=1, K=2, N=36, N_fft=64, L=4.0, slots=3, snr=10.0),               # 3 tones: the minimum
    dict(M=1, K=1, N=24576, N_fft=32768, L=8.0, slots=1, snr=20.0),         # 2048 tones: spline maximum
]


@pytest.mark.parametrize("kind", ["ls_quadratic", "ls_spline"])
@pytest.mark.parametrize("c", [CASES[0], CASES[1], CASES[2], CASES[5]] + EDGE_LS)
def test_higher_order_interpolated_ls_match_oracle(dev, c, kind):
    print(f"comb {kind} {c}", flush=True)
    S = c.get("comb", 12)
    cb = make_comb_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], powers_db=PROFILE,
                         snr_db=c["snr"], slots=c["slots"], comb=S)
    with _plan(c, kind, cb.sigma2) as pl:
        out = pl.estimate(_t(cb.y, dev), _t(cb.pilots, dev)).cpu().numpy()
    f = O.comb_ls_quadratic if kind == "ls_quadratic" else O.comb_ls_spline
    ref = f(cb.y, cb.pilots, S, range(c["K"]))
    disc = O.discrepancy_db(out, ref)
    print(f"  discrepancy {disc:.1f} dB", flush=True)
    assert disc < -120.0
