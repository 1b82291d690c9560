"""GPU gradients of the sample-covariance estimator (the filter of every
(slot, user, window) designed from that window's own covariance) against
the FP64 oracle's hand-derived gradients, FP64 central finite differences of
the oracle loss in sigma2 (relative step 1e-4), through the C ABI and
through SampleLmmseFn.  Both sides read the same complex64 LS values, the
oracle's despreading of seeded synthetic slots."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import Plan
from paper_1802_05427_amd.autograd import SampleLmmseFn
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


def _oracle_estimate(X, B, Wn, sigma2):
    """Sample-covariance estimate, block by block (eq. 13 on each window)."""
    S, M, K, N = X.shape
    lam = sigma2 / K
    out = np.zeros_like(X)
    starts, offs = O.window_starts(N, B, Wn)
    for s in range(S):
        for k in range(K):
            for b, (st, off) in enumerate(zip(starts, offs)):
                Xw = X[s, :, k, st:st + Wn]
                R = O.sample_covariance(Xw)
                W = O.lmmse._filter(R[off:off + B], R, lam)
                out[s, :, k, b * B:(b + 1) * B] = Xw @ W.T
    return out


CASES = [
    dict(M=8, K=2, N=72, N_fft=128, taps=8, tau=2.0, B=12, Wn=24, slots=2),      # overlap, M < Wn
    dict(M=6, K=2, N=72, N_fft=128, taps=8, tau=3.0, B=12, Wn=12, slots=2),      # non-overlapping
    dict(M=6, K=3, N=99, N_fft=128, taps=8, tau=2.0, B=9, Wn=21, slots=3),       # odd B, odd Wn
    dict(M=70, K=2, N=240, N_fft=256, taps=12, tau=3.0, B=60, Wn=120, slots=1),  # several GEMM tiles
    dict(M=20, K=3, N=1200, N_fft=2048, taps=72, tau=4.0, B=100, Wn=150, slots=1),
    # wider than the register-resident design: 7 sweep panels in the workspace
    dict(M=20, K=2, N=400, N_fft=512, taps=16, tau=4.0, B=100, Wn=200, slots=2),
]


@pytest.mark.parametrize("c", CASES)
def test_sample_backward_matches_oracle_and_fd(dev, c):
    print(f"sample backward {c}", flush=True)
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=4)
    B, Wn, sig = c["B"], c["Wn"], 0.05
    X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
    X = X32.astype(np.complex128)
    L0, G = O.mse_loss_and_grad(_oracle_estimate(X, B, Wn, sig), sb.H)
    G32 = G.astype(np.complex64)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=B, Wn=Wn, rsource="sample",
              sigma2=sig, max_slots=c["slots"]) as plan:
        plan.set_design(float("nan"), sig)
        d_hls, d_tau, d_sig = plan.backward(_t(X32, dev), _t(G32, dev))
        st, info = plan.sync_status()
        d_hls = d_hls.cpu().numpy()
    assert st == 0, (st, info)
    dX_o, gsig_o = O.grad_sample_cov(X, G32.astype(np.complex128), B, Wn, sig)
    ex = np.linalg.norm(d_hls - dX_o) / np.linalg.norm(dX_o)
    print(f"  dX rel {ex:.2e}  dsig gpu {d_sig:.8e} oracle {gsig_o:.8e}", flush=True)
    assert np.isnan(d_tau)
    assert ex < 1e-5
    assert abs(d_sig - gsig_o) <= 1e-6 * abs(gsig_o)
    hh = 1e-4
    fd = (O.mse_loss_and_grad(_oracle_estimate(X, B, Wn, sig * (1 + hh)), sb.H)[0]
          - O.mse_loss_and_grad(_oracle_estimate(X, B, Wn, sig * (1 - hh)), sb.H)[0]) / (2 * hh * sig)
    assert abs(d_sig - fd) <= REL * abs(fd)


def test_sample_backward_is_not_the_fixed_formula(dev):
    """The filter depends on h_ls through R: W^H G alone differs from the gradient."""
    c = CASES[0]
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=1, config_id=4)
    X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
    G32 = (np.random.default_rng(5).standard_normal(X32.shape)
           + 1j * np.random.default_rng(6).standard_normal(X32.shape)).astype(np.complex64)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="sample",
              sigma2=0.05, max_slots=1) as plan:
        plan.set_design(float("nan"), 0.05)
        d_hls = plan.backward(_t(X32, dev), _t(G32, dev), want_params=False)[0].cpu().numpy()
    X = X32.astype(np.complex128)
    G = G32.astype(np.complex128)
    lam = 0.05 / c["K"]
    starts, offs = O.window_starts(c["N"], c["B"], c["Wn"])
    fixed_only = np.zeros_like(X)
    for k in range(c["K"]):
        for b, (st, off) in enumerate(zip(starts, offs)):
            Xw = X[0, :, k, st:st + c["Wn"]]
            R = O.sample_covariance(Xw)
            W = O.lmmse._filter(R[off:off + c["B"]], R, lam)
            fixed_only[0, :, k, st:st + c["Wn"]] += G[0, :, k, b * c["B"]:(b + 1) * c["B"]] @ np.conj(W)
    dX_o, _ = O.grad_sample_cov(X, G, c["B"], c["Wn"], 0.05)
    assert np.linalg.norm(d_hls - dX_o) < 1e-5 * np.linalg.norm(dX_o)
    assert np.linalg.norm(d_hls - fixed_only) > 1e-3 * np.linalg.norm(dX_o)


def test_sample_autograd_function(dev):
    c = CASES[2]
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=4)
    X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
    X = X32.astype(np.complex128)
    H32 = sb.H.astype(np.complex64)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="sample",
              sigma2=0.05, max_slots=c["slots"]) as plan:
        h = _t(X32, dev).requires_grad_(True)
        sig = torch.tensor(0.03, dtype=torch.float64, requires_grad=True)
        out = SampleLmmseFn.apply(h, sig, plan)
        loss = (out - _t(H32, dev)).abs().pow(2).sum() / out.numel()
        loss.backward()
        est = out.detach().cpu().numpy()
    ref = _oracle_estimate(X, c["B"], c["Wn"], 0.03)
    L0, G = O.mse_loss_and_grad(ref, H32.astype(np.complex128))
    dX_o, gsig_o = O.grad_sample_cov(X, G, c["B"], c["Wn"], 0.03)
    assert O.discrepancy_db(est, ref) < -100
    assert abs(float(loss.detach()) - L0) <= 1e-5 * L0
    assert abs(float(sig.grad) - gsig_o) <= 1e-3 * abs(gsig_o)
    ex = np.linalg.norm(h.grad.cpu().numpy() - dX_o) / np.linalg.norm(dX_o)
    assert ex < 1e-4


KEEP_CASES = [
    # FP32 matrix-core covariance in the resident design (windows 161..208)
    dict(M=40, K=2, N=396, N_fft=512, taps=16, tau=4.0, B=132, Wn=198, slots=1),
    # FP64 matrix-core covariance (windows 129..160), two slots
    dict(M=24, K=2, N=400, N_fft=512, taps=16, tau=4.0, B=100, Wn=150, slots=2),
]


@pytest.mark.parametrize("c", KEEP_CASES)
def test_kept_design_backward_matches_recomputed(dev, c):
    """lmmse_estimate_ls_keep / lmmse_backward_kept: the forward's output and the
    backward's d_hls and parameter gradients equal those of the calls that form
    the design again, bit for bit (twice: the state is only read), and the kept
    gradients meet the oracle bars of the recomputing backward."""
    print(f"kept design {c}", flush=True)
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=4)
    B, Wn, sig, S = c["B"], c["Wn"], 0.05, c["slots"]
    X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
    X = X32.astype(np.complex128)
    _, G = O.mse_loss_and_grad(_oracle_estimate(X, B, Wn, sig), sb.H)
    G32 = G.astype(np.complex64)
    h, g = _t(X32, dev), _t(G32, dev)
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=B, Wn=Wn, rsource="sample",
              sigma2=sig, max_slots=S) as plan:
        nbytes = plan.design_state_bytes(S)
        assert nbytes == S * c["K"] * (c["N"] // B) * (B * Wn + Wn * Wn) * 16
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        o_plain = plan.estimate_ls(h, sig)
        o_keep = plan.estimate_ls(h, sig, keep=state)
        p = [torch.empty(2, dtype=torch.float64, device=dev) for _ in range(3)]
        d1, _, _ = plan.backward(h, g, params_out=p[0])
        d2, _, _ = plan.backward(h, g, params_out=p[1], kept=state)
        d3, _, _ = plan.backward(h, g, params_out=p[2], kept=state)
        st, info = plan.sync_status()
    assert st == 0, (st, info)
    assert torch.equal(o_plain, o_keep)
    assert torch.equal(d1, d2) and torch.equal(d2, d3)
    a = [t.cpu().numpy() for t in p]
    np.testing.assert_array_equal(a[0], a[1])
    np.testing.assert_array_equal(a[1], a[2])
    dX_o, gsig_o = O.grad_sample_cov(X, G32.astype(np.complex128), B, Wn, sig)
    ex = np.linalg.norm(d2.cpu().numpy() - dX_o) / np.linalg.norm(dX_o)
    print(f"  dX rel {ex:.2e}  dsig gpu {a[1][1]:.8e} oracle {gsig_o:.8e}", flush=True)
    assert np.isnan(a[1][0])
    assert ex < 1e-5
    assert abs(a[1][1] - gsig_o) <= 1e-6 * abs(gsig_o)


def test_sample_autograd_function_kept_design(dev):
    """SampleLmmseFn with keep=True: the same estimate and gradients, bit for
    bit, as with the design formed again in the backward."""
    c = KEEP_CASES[1]
    sb = make_slot_batch(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], taps=c["taps"], tau=c["tau"],
                         snr_db=10.0, slots=c["slots"], config_id=4)
    X32 = O.despread(sb.y, sb.pilots).astype(np.complex64)
    H = _t(sb.H.astype(np.complex64), dev)
    res = []
    with Plan(M=c["M"], K=c["K"], N=c["N"], N_fft=c["N_fft"], B=c["B"], Wn=c["Wn"], rsource="sample",
              sigma2=0.05, max_slots=c["slots"]) as plan:
        assert plan.design_state_bytes(c["slots"]) > 0
        for keep in (False, True):
            h = _t(X32, dev).requires_grad_(True)
            sig = torch.tensor(0.03, dtype=torch.float64, requires_grad=True)
            out = SampleLmmseFn.apply(h, sig, plan, keep)
            loss = (out - H).abs().pow(2).sum() / out.numel()
            loss.backward()
            res.append((out.detach(), h.grad.detach(), sig.grad.detach()))
    assert torch.equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1], res[1][1])
    assert torch.equal(res[0][2], res[1][2])


def test_kept_design_needs_a_resident_window(dev):
    """Windows the register-resident design holds (here 120) keep no state:
    size 0, and the keeping calls refuse the plan."""
    from paper_1802_05427_amd._lib import LmmseError
    with Plan(M=8, K=2, N=240, N_fft=256, B=60, Wn=120, rsource="sample", sigma2=0.05,
              max_slots=1) as plan:
        assert plan.design_state_bytes(1) == 0
        h = torch.zeros(1, 8, 2, 240, dtype=torch.complex64, device=dev)
        with pytest.raises(LmmseError):
            plan.estimate_ls(h, 0.05, keep=torch.empty(256, dtype=torch.uint8, device=dev))


def test_kept_design_error_paths(dev):
    """The keeping calls through the C ABI: a state shorter than
    lmmse_design_state_size is LMMSE_ERR_WORKSPACE and a missing one
    LMMSE_ERR_INVALID_ARG (nothing launched), and a fixed-design plan keeps
    nothing (size 0, LMMSE_ERR_UNSUPPORTED)."""
    import ctypes

    from paper_1802_05427_amd import _lib
    P = lambda t: ctypes.c_void_p(t.data_ptr())   # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    h = torch.zeros(1, 24, 2, 400, dtype=torch.complex64, device=dev)
    out = torch.empty_like(h)
    par = torch.empty(2, dtype=torch.float64, device=dev)
    with Plan(M=24, K=2, N=400, N_fft=512, B=100, Wn=150, rsource="sample", sigma2=0.05,
              max_slots=1) as plan:
        lib = plan._lib
        need = plan.design_state_bytes(1)
        assert need > 0
        short = torch.empty(need - 256, dtype=torch.uint8, device=dev)
        ws, wsb = plan._workspace(1)
        assert lib.lmmse_estimate_ls_keep(plan._h, 1, P(h), 0.05, P(out), P(short), need - 256, ws, wsb,
                                          stream) == _lib.WORKSPACE
        assert lib.lmmse_estimate_ls_keep(plan._h, 1, P(h), 0.05, P(out), None, 0, ws, wsb,
                                          stream) == _lib.INVALID_ARG
        assert lib.lmmse_backward_kept(plan._h, 1, P(h), P(h), P(out), P(par), P(short), need - 256, ws,
                                       wsb, stream) == _lib.WORKSPACE
        assert lib.lmmse_backward_kept(plan._h, 1, P(h), P(h), P(out), P(par), None, 0, ws, wsb,
                                       stream) == _lib.INVALID_ARG
    with Plan(M=24, K=2, N=400, N_fft=512, B=100, Wn=150, rsource="exp", taps=16, tau_rms=4.0,
              sigma2=0.05, max_slots=1) as fixed:
        assert fixed.design_state_bytes(1) == 0
        big = torch.empty(need, dtype=torch.uint8, device=dev)
        ws, wsb = fixed._workspace(1)
        assert fixed._lib.lmmse_backward_kept(fixed._h, 1, P(h), P(h), P(out), P(par), P(big), need, ws,
                                              wsb, stream) == _lib.UNSUPPORTED
    torch.cuda.synchronize()
