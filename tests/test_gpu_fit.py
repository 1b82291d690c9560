"""Adam fit of the fixed exponential design on simulated MSE (GPU).

With channels drawn at one delay spread, the expected error is stationary at
the true (tau_rms, sigma2) (the exponential design family contains the
matched filters), so the fit must move towards them; with the spread drawn
per (slot, user) from U[2, 24] at the differentiation workload's shape, it
must end at the FP64 oracle's minimiser of the expected error; and a fit
resumed from a saved state must retrace the uninterrupted trajectory
exactly."""
import math
import os

import pytest
import torch

from paper_1802_05427_amd import Plan
from paper_1802_05427_amd.fit import FitState, fit_design
from synth import make_pilots
from synth.torch_slots import draw_batch

pytestmark = pytest.mark.gpu

CFG = dict(M=16, K=4, N=240, N_fft=256, taps=24, B=40, Wn=60, slots=4)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _batch_fn(plan, dev, tau_true, sigma2, seed):
    c = CFG
    pil = torch.from_numpy(make_pilots(c["K"], c["N"])).to(dev)

    def fn(step):
        g = torch.Generator(device=dev)
        g.manual_seed(seed * 100003 + step)
        y, H, _ = draw_batch(g, c["slots"], c["M"], c["K"], c["N"], c["N_fft"], c["taps"], tau_true,
                             tau_true, sigma2, pil)
        return plan.despread(y, pil), H

    return fn


def _plan():
    c = CFG
    return Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="exp",
                taps=c["taps"], tau_rms=8.0, sigma2=1e-4, max_slots=c["slots"])


def test_fit_moves_to_true_design(dev):
    tau_true, sig_true = 3.0, 0.1
    with _plan() as plan:
        st = fit_design(plan, _batch_fn(plan, dev, tau_true, sig_true, 1), steps=150, lr=0.08,
                        tau0=8.0, sigma2_0=1e-3)
    h = st.history
    first = sum(x[0] for x in h[:10]) / 10
    last = sum(x[0] for x in h[-10:]) / 10
    tau_f, sig_f = h[-1][1], h[-1][2]
    print(f"loss {first:.4e} -> {last:.4e}; tau {tau_f:.3f} (true {tau_true}); sigma2 {sig_f:.4f}", flush=True)
    assert last < first
    # measured: tau 3.024, sigma2 0.1037
    assert abs(tau_f - tau_true) / tau_true < 0.05
    assert 0.8 < sig_f / sig_true < 1.25


def test_fit_resume_is_exact(dev, tmp_path):
    with _plan() as plan:
        fn = _batch_fn(plan, dev, 4.0, 0.05, 2)
        full = fit_design(plan, fn, steps=12, lr=0.05)
        half = fit_design(plan, fn, steps=6, lr=0.05)
        path = os.path.join(tmp_path, "fit.json")
        half.save(path)
        resumed = fit_design(plan, fn, steps=12, lr=0.05, state=FitState.load(path))
    for a, b in zip(full.history, resumed.history):
        assert a == b
    assert math.isclose(full.log_tau, resumed.log_tau, rel_tol=0, abs_tol=0)


# The differentiation workload itself: M=128, K=12, N=1200 of 2048,
# overlapping windows of 150 keeping 100, 72 taps, 16 slots per batch with
# tau_rms ~ U[2, 24] per (slot, user), SNR 10 dB, 200 Adam steps from
# tau = 8, sigma2 = 1e-4 (lr 0.05).  The endpoint is compared with the FP64
# oracle's minimiser of the expected error over the design (stored by
# tests/golden/make_fit_optimum.py): the expected error of the fitted design
# is evaluated by the oracle's closed form at the spread-averaged correlation.
DIFF = dict(M=128, K=12, N=1200, N_fft=2048, taps=72, B=100, Wn=150, slots=16, sigma2=0.1)


def test_fit_reaches_oracle_optimum_at_differentiation_workload(dev, golden_dir):
    import json

    import numpy as np

    import oracle as O
    from oracle.fit_optimum import design_mse, mixture_r

    c = DIFF
    with open(os.path.join(golden_dir, "fit_optimum_diff_workload.json")) as f:
        opt = json.load(f)
    pil = torch.from_numpy(make_pilots(c["K"], c["N"])).to(dev)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="exp",
              taps=c["taps"], tau_rms=8.0, sigma2=1e-4, max_slots=c["slots"]) as plan:
        def fn(step):
            g = torch.Generator(device=dev)
            g.manual_seed(180205427 + 7919 * step)
            y, H, _ = draw_batch(g, c["slots"], c["M"], c["K"], c["N"], c["N_fft"], c["taps"], 2.0,
                                 24.0, c["sigma2"], pil)
            return plan.despread(y, pil), H

        st = fit_design(plan, fn, steps=200, lr=0.05, tau0=8.0, sigma2_0=1e-4)
    # the endpoint: the mean of the last 20 iterates (Adam jitters around it)
    tail = np.array(st.history[-20:])
    tau_f, sig_f = float(np.exp(np.log(tail[:, 1]).mean())), float(np.exp(np.log(tail[:, 2]).mean()))
    n = np.arange(c["N"])
    Rb = O.toeplitz_from_r(lambda d: mixture_r(d, 2.0, 24.0, c["taps"], c["N_fft"]), n, n)
    lam = c["sigma2"] / c["K"]
    e_fit = design_mse(tau_f, sig_f, Rb, lam, c["B"], c["Wn"], c["K"], c["taps"], c["N_fft"])
    e_start = design_mse(8.0, 1e-4, Rb, lam, c["B"], c["Wn"], c["K"], c["taps"], c["N_fft"])
    excess_db = 10 * np.log10(e_fit / opt["mse"])
    start_db = 10 * np.log10(e_start / opt["mse"])
    print(f"fit endpoint tau {tau_f:.3f} sigma2 {sig_f:.4f} (oracle optimum {opt['tau']:.3f}, "
          f"{opt['sigma2']:.4f}); expected error {excess_db:.4f} dB above the optimum "
          f"(start {start_db:.3f} dB); last loss {st.history[-1][0]:.4e}", flush=True)
    # the start is 0.54 dB above the optimum; the surface is flat near it
    # (tau off by 10 % costs 0.005-0.011 dB, sigma2 off by 2x 0.03-0.05 dB).
    # Measured: 0.0003 dB, tau 14.27 against 14.42, sigma2 0.0887 against 0.0858.
    assert excess_db < 0.005
    assert abs(tau_f - opt["tau"]) / opt["tau"] < 0.06
    assert 0.8 < sig_f / opt["sigma2"] < 1.25
