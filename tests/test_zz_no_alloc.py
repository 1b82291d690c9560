"""lmmse_estimate_noalloc (the estimate on the library's static device
workspace) against lmmse_estimate with a caller workspace, through the C ABI:
two calls in a row on one plan, the second with fewer slots, for the paths
that use a workspace (sample covariance: H_LS and per-window filters; a user
count the fused kernel does not take: H_LS staging) and for the fused path
(no workspace).  Requests beyond the static size are refused before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import Plan, _lib
from synth import make_slot_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    # (M, K, N, N_fft, taps, tau, B, Wn, rsource, precision)
    (16, 4, 240, 256, 24, 3.0, 40, 60, "sample", "fp32"),
    (16, 4, 240, 256, 24, 3.0, 40, 60, "sample", "bf16x3"),
    (12, 3, 120, 128, 12, 2.0, 24, 36, "exp", "fp32"),      # K = 3: despread, then filter
    (16, 4, 240, 256, 24, 3.0, 40, 60, "exp", "fp32"),      # fused, no workspace
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[8]}-K{c[1]}-{c[9]}")
def test_noalloc_matches_workspace_estimate(dev, case):
    M, K, N, Nf, taps, tau, B, Wn, rs, prec = case
    S = 4
    sb = make_slot_batch(M=M, K=K, N=N, N_fft=Nf, taps=taps, tau=tau, snr_db=10.0, slots=S, config_id=90)
    y = torch.from_numpy(sb.y).to(dev)
    pil = torch.from_numpy(sb.pilots).to(dev)
    print(f"noalloc case {case}", flush=True)
    with Plan(M=M, K=K, N=N, N_fft=Nf, B=B, Wn=Wn, rsource=rs, taps=taps, tau_rms=tau, sigma2=sb.sigma2,
              max_slots=S, precision=prec) as plan:
        for ns in (S, S // 2):   # second call with a smaller input
            ref = plan.estimate(y[:ns].contiguous(), pil, sb.sigma2)
            out = torch.full_like(ref, float("nan"))
            plan.estimate_noalloc(y[:ns].contiguous(), pil, sb.sigma2, out=out)
            torch.cuda.synchronize()
            r, o = ref.cpu().numpy(), out.cpu().numpy()
            assert np.all(np.isfinite(o))
            # the same kernels on the same inputs: agreement to the FP32 bar
            # (discrepancy below -120 dB; measured bit-identical)
            d = O.discrepancy_db(o, r) if np.any(o != r) else -np.inf
            print(f"  slots {ns}: discrepancy vs workspace estimate {d} dB", flush=True)
            assert d < -120.0
            if rs != "sample":
                ora = O.estimate(sb.y[:ns], sb.pilots, sb.sigma2, B, Wn, rs, N_fft=Nf, tau=tau, taps=taps)
                assert O.discrepancy_db(o, ora) < -100.0


def test_noalloc_refuses_oversized_request(dev):
    # sample covariance on 4 paper-sized slots needs about 128 MB of workspace
    M, K, N, Nf, B, Wn, S = 128, 12, 1200, 2048, 100, 150, 4
    with Plan(M=M, K=K, N=N, N_fft=Nf, B=B, Wn=Wn, rsource="sample", sigma2=0.1, max_slots=S) as plan:
        assert plan.workspace_bytes(S) > _lib.NOALLOC_SCRATCH_BYTES
        y = torch.zeros((S, M, K, N), dtype=torch.complex64, device=dev)
        pil = torch.ones((K, N), dtype=torch.complex64, device=dev)
        out = torch.zeros_like(y)
        lib = _lib.load()
        rc = lib.lmmse_estimate_noalloc(plan._h, S, ctypes.c_void_p(y.data_ptr()),
                                        ctypes.c_void_p(pil.data_ptr()), 0.1,
                                        ctypes.c_void_p(out.data_ptr()), None)
        assert rc == _lib.WORKSPACE
        # one slot fits
        plan.estimate_noalloc(y[:1].contiguous(), pil, 0.1, out=out[:1])
        torch.cuda.synchronize()
        assert torch.all(out[1:] == 0)
