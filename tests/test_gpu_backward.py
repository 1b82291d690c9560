"""GPU gradients of the fixed exponential design against the FP64 oracle's
hand-derived gradients and against FP64 central finite differences
(relative step 1e-4), through the C ABI and through LmmseFn."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import Plan
from paper_1802_05427_amd.autograd import LmmseFn
from synth import make_slot_batch

pytestmark = pytest.mark.gpu

REL = 1e-3      # gradients within 1e-3 relative of finite differences


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _oracle_loss(X, H, B, Wn, tau, taps, N_fft, sigma2, K):
    n = np.arange(X.shape[-1])
    R = O.toeplitz_from_r(lambda d: O.r_exponential(d, tau, taps, N_fft), n, n)
    Ws, st = O.block_filters(R, B, Wn, sigma2 / K)
    return O.mse_loss_and_grad(O.apply_filters(Ws, st, B, X), H)


CASES = [
    dict(M=6, K=2, N=72, N_fft=128, taps=8, tau=3.0, B=12, Wn=24, slots=2, design_tau=4.5),
    dict(M=6, K=2, N=72, N_fft=128, taps=8, tau=3.0, B=12, Wn=12, slots=1, design_tau=2.0),
    dict(M=5, K=3, N=96, N_fft=128, taps=8, tau=2.0, B=16, Wn=48, slots=1, design_tau=3.0),
    dict(M=6, K=3, N=99, N_fft=128, taps=8, tau=2.0, B=9, Wn=21, slots=2, design_tau=3.0),
    dict(M=16, K=12, N=1200, N_fft=2048, taps=72, tau=4.0, B=100, Wn=150, slots=1, design_tau=8.0),
    # large system: 2B = 264 real rows (three dW row groups), 13 window tiles
    dict(M=2, K=24, N=3300, N_fft=4096, taps=144, tau=32.0, B=132, Wn=198, slots=1, design_tau=24.0),
    # four passes whose first leaves 75 runs of subcarriers uncovered: dX is
    # zeroed whole and every pass adds
    dict(M=2, K=2, N=1200, N_fft=2048, taps=8, tau=3.0, B=4, Wn=10, slots=1, design_tau=4.0),
]


@pytest.mark.parametrize("c", CASES)
def test_backward_matches_oracle_and_fd(dev, c):
    print(f"backward {c}", flush=True)
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=3)
    K, tau, sig = c["K"], c["design_tau"], 1e-2
    args = (c["B"], c["Wn"], tau, c["taps"], c["N_fft"], sig, K)
    with Plan(M=c["M"], K=K, N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="exp",
              taps=c["taps"], tau_rms=tau, sigma2=sig, max_slots=c["slots"]) as plan:
        # the same complex64 LS values (the oracle's despreading) feed both sides
        X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
        h = _t(X32, dev)
        X = X32.astype(np.complex128)
        L0, G = _oracle_loss(X, sb.H, *args)
        d_hls, d_tau, d_sig = plan.backward(h, _t(G.astype(np.complex64), dev))
        d_hls = d_hls.cpu().numpy()
    dX_o, gtau_o, gsig_o = O.grad_fixed_design(X, G.astype(np.complex64).astype(np.complex128),
                                               c["B"], c["Wn"], tau, c["taps"], c["N_fft"], sig, K)
    ex = np.linalg.norm(d_hls - dX_o) / np.linalg.norm(dX_o)
    print(f"  dX rel {ex:.2e}  dtau gpu {d_tau:.6e} oracle {gtau_o:.6e}  dsig gpu {d_sig:.6e} oracle {gsig_o:.6e}",
          flush=True)
    assert ex < 1e-5
    assert abs(d_tau - gtau_o) <= 1e-4 * abs(gtau_o)
    assert abs(d_sig - gsig_o) <= 1e-4 * abs(gsig_o)
    # FP64 central differences of the oracle loss, relative step 1e-4
    hh = 1e-4
    fd_tau = (_oracle_loss(X, sb.H, c["B"], c["Wn"], tau * (1 + hh), c["taps"], c["N_fft"], sig, K)[0]
              - _oracle_loss(X, sb.H, c["B"], c["Wn"], tau * (1 - hh), c["taps"], c["N_fft"], sig, K)[0]) \
        / (2 * hh * tau)
    fd_sig = (_oracle_loss(X, sb.H, c["B"], c["Wn"], tau, c["taps"], c["N_fft"], sig * (1 + hh), K)[0]
              - _oracle_loss(X, sb.H, c["B"], c["Wn"], tau, c["taps"], c["N_fft"], sig * (1 - hh), K)[0]) \
        / (2 * hh * sig)
    assert abs(d_tau - fd_tau) <= REL * abs(fd_tau)
    assert abs(d_sig - fd_sig) <= REL * abs(fd_sig)


def test_autograd_function(dev):
    c = CASES[0]
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=3)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="exp",
              taps=c["taps"], tau_rms=4.0, sigma2=0.05, max_slots=c["slots"]) as plan:
        X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
        h = _t(X32, dev).requires_grad_(True)
        tau = torch.tensor(4.5, dtype=torch.float64, requires_grad=True)
        sig = torch.tensor(0.02, dtype=torch.float64, requires_grad=True)
        H = _t(sb.H.astype(np.complex64), dev)
        out = LmmseFn.apply(h, tau, sig, plan)
        loss = (out - H).abs().pow(2).sum() / out.numel()
        loss.backward()
        X = X32.astype(np.complex128)
        L0, G = _oracle_loss(X, sb.H.astype(np.complex64).astype(np.complex128), c["B"], c["Wn"], 4.5,
                             c["taps"], c["N_fft"], 0.02, c["K"])
        dX_o, gtau_o, gsig_o = O.grad_fixed_design(X, G, c["B"], c["Wn"], 4.5, c["taps"], c["N_fft"], 0.02,
                                                   c["K"])
    assert abs(float(loss.detach()) - L0) <= 1e-5 * L0
    assert abs(float(tau.grad) - gtau_o) <= 1e-3 * abs(gtau_o)
    assert abs(float(sig.grad) - gsig_o) <= 1e-3 * abs(gsig_o)
    ex = np.linalg.norm(h.grad.cpu().numpy() - dX_o) / np.linalg.norm(dX_o)
    assert ex < 1e-4


@pytest.mark.parametrize("rsource", ["exp", "uniform"])
def test_backward_device_params_match_host(dev, rsource):
    """lmmse_backward_dev leaves d_tau / d_sigma2 on the device: the same
    d_hls and the same two scalars (NaN where the host call gives NaN) as
    lmmse_backward, bit for bit, on two calls in a row."""
    c = dict(M=16, K=12, N=1200, N_fft=2048, taps=72, tau=4.0, B=100, Wn=150, slots=2)
    print(f"device params {rsource} {c}", flush=True)
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=3)
    kw = dict(rsource=rsource, taps=c["taps"], tau_rms=6.0) if rsource == "exp" else dict(rsource=rsource, L=144.0)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], sigma2=1e-2,
              max_slots=c["slots"], **kw) as plan:
        h = _t(O.despread(sb.y, sb.pilots).astype(np.complex64), dev)
        g = _t((sb.H * (2.0 / sb.H.size)).astype(np.complex64), dev)
        dx_h, t_h, s_h = plan.backward(h, g)
        par = torch.full((2,), 7.0, dtype=torch.float64, device=dev)
        for _ in range(2):
            dx_d, t_d, s_d = plan.backward(h, g, params_out=par)
            torch.cuda.synchronize()
            assert torch.equal(dx_d, dx_h)
            got = par.cpu().numpy()
            for gv, hv in zip(got, (t_h, s_h)):
                assert (np.isnan(gv) and np.isnan(hv)) or gv == hv, (got, t_h, s_h)
            par.fill_(7.0)
    assert np.isfinite(s_h)
    assert np.isfinite(t_h) == (rsource == "exp")
