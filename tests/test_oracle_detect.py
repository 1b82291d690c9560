"""Pins of the MMSE detection oracle (eq. 20-22): the push-through identity
(a different matrix: the M x M form), the noiseless zero-forcing limit, and
correct QPSK decisions at high SNR."""
import numpy as np

import oracle as O
from synth import make_data_symbols, make_slot_batch


def _H(M=8, K=3, N=24, S=2):
    return make_slot_batch(M=M, K=K, N=N, N_fft=64, taps=4, tau=2.0, snr_db=None, slots=S,
                           config_id=6).H


def test_push_through_identity():
    """(H^H H + s I)^-1 H^H Y = H^H (H H^H + s I)^-1 Y, the right side from the
    M x M system solved by np.linalg.solve."""
    H = _H()
    Y, _, _ = make_data_symbols(H, T=5, snr_db=5.0)
    s2 = 0.3
    X = O.mmse_detect(H, Y, s2)
    S, M, K, N = H.shape
    for s in range(S):
        for n in range(N):
            h = H[s, :, :, n]
            ref = np.conj(h).T @ np.linalg.solve(h @ np.conj(h).T + s2 * np.eye(M),
                                                 Y[s, :, :, n].astype(np.complex128))
            assert np.allclose(X[s, :, :, n], ref.T, atol=1e-10)


def test_noiseless_limit_recovers_the_symbols():
    H = _H(M=10, K=4)
    Y, X, _ = make_data_symbols(H, T=3, snr_db=None)
    Xh = O.mmse_detect(H, Y, 1e-9)
    assert np.abs(Xh - X).max() < 1e-5


def test_high_snr_decisions():
    H = _H(M=16, K=4, N=48, S=1)
    Y, X, s2 = make_data_symbols(H, T=4, snr_db=25.0)
    Xh = O.mmse_detect(H, Y, s2)
    assert np.mean(O.qpsk_decide(Xh) != X) < 1e-3
