"""Adam fit of the fixed exponential design on simulated MSE (GPU).

With channels drawn at one delay spread, the expected error is stationary at
the true (tau_rms, sigma2) (the exponential design family contains the
matched filters), so the fit must move towards them; and a fit resumed from
a saved state must retrace the uninterrupted trajectory exactly."""
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
    assert abs(tau_f - tau_true) / tau_true < 0.15
    assert 0.25 < sig_f / sig_true < 4.0


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
