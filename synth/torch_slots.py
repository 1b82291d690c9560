"""The slot generator of slots.py drawn on the GPU with torch (inputs only).

Same model: integer-delay taps h_l ~ CN(0, p_l) with an exponential profile,
H[n] = sum_l h_l exp(-j 2 pi l n / N_fft) over the contiguous bins 0..N-1,
user k sends c[k,t] x_k[n] on pilot symbol t with the DFT cover
c[k,t] = exp(-j 2 pi k t / K), noise CN(0, sigma2).  Used where a fresh batch
per optimisation step is needed (the design fit): drawing 16 paper-sized
slots on the host would dominate the step.  Seeded with a torch.Generator on
the device; the streams differ from slots.py's NumPy streams.
"""
from __future__ import annotations

import math

import torch


def draw_batch(gen: torch.Generator, slots: int, M: int, K: int, N: int, N_fft: int, taps: int,
               tau_lo: float, tau_hi: float, sigma2: float, pilots: torch.Tensor):
    """Returns (y [S,M,K,N] c64, H [S,M,K,N] c64, tau [S,K] f64) on pilots.device."""
    dev = pilots.device
    tau = tau_lo + (tau_hi - tau_lo) * torch.rand((slots, K), generator=gen, device=dev,
                                                  dtype=torch.float64)
    l = torch.arange(taps, device=dev, dtype=torch.float64)
    w = torch.exp(-l[None, None, :] / tau[:, :, None])            # [S,K,L]
    p = w / w.sum(-1, keepdim=True)
    std = torch.sqrt(p / 2.0).to(torch.float32)[:, None]          # [S,1,K,L]
    re = torch.randn((slots, M, K, taps), generator=gen, device=dev)
    im = torch.randn((slots, M, K, taps), generator=gen, device=dev)
    h = torch.complex(re * std, im * std)
    H = torch.fft.fft(h, n=N_fft, dim=-1)[..., :N].contiguous()
    v = H * pilots[None, None]
    y = torch.fft.fft(v, dim=2)
    if sigma2 > 0:
        s = math.sqrt(sigma2 / 2.0)
        y = y + torch.complex(torch.randn(y.shape, generator=gen, device=dev) * s,
                              torch.randn(y.shape, generator=gen, device=dev) * s)
    return y.to(torch.complex64).contiguous(), H.to(torch.complex64), tau
