"""GPU parity of MMSE MIMO detection (eq. 22) against the FP64 oracle on
seeded channels and QPSK data symbols: ragged antenna and subcarrier counts,
K and T from 1 to the limit of 16, and detection on the estimator's own
output layout."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1802_05427_amd import mmse_detect
from synth import make_data_symbols, make_slot_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("M,K,T,N,S,snr", [
    (8, 2, 3, 40, 2, 10.0),      # N not a multiple of 16
    (13, 4, 1, 48, 1, 15.0),     # M not a multiple of 8, one data symbol
    (128, 12, 12, 96, 1, 10.0),  # paper-sized antennas and users
    (32, 16, 16, 33, 2, 20.0),   # K and T at the limit
    (16, 1, 16, 17, 1, 5.0),     # one user
])
def test_detect_matches_oracle(dev, M, K, T, N, S, snr):
    print(f"detect M={M} K={K} T={T} N={N} S={S}", flush=True)
    H = make_slot_batch(M=M, K=K, N=N, N_fft=128, taps=6, tau=2.0, snr_db=None, slots=S,
                        config_id=7).H.astype(np.complex64)
    Y, X, s2 = make_data_symbols(H.astype(np.complex128), T=T, snr_db=snr)
    got = mmse_detect(_t(H, dev), _t(Y, dev), s2).cpu().numpy()
    ref = O.mmse_detect(H.astype(np.complex128), Y.astype(np.complex128), s2)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  relative error {err:.2e}", flush=True)
    assert np.isfinite(got).all()
    assert err < 1e-5


def test_detect_rejects_too_many_users(dev):
    from paper_1802_05427_amd import LmmseError
    h = torch.zeros((1, 20, 17, 16), dtype=torch.complex64, device=dev)
    y = torch.zeros((1, 20, 2, 16), dtype=torch.complex64, device=dev)
    with pytest.raises(LmmseError):
        mmse_detect(h, y, 0.1)
