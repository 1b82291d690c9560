"""Gradient fit of the fixed design's assumed delay spread and noise variance.

The paper tunes its assumed channel length by measured BER (Sec. IV-C); here
the exponential design (tau_rms, sigma2) is fitted by Adam on the simulated
MSE of the partitioned estimator, with gradients from lmmse_backward (via
LmmseFn).  Parameters are optimised in log space; each step draws a fresh
batch of slots.  The state (parameters, Adam moments, step, seed) can be
saved and restored so that a resumed fit follows the same trajectory.
"""
from __future__ import annotations

import json
import math
from dataclasses import asdict, dataclass, field

import torch

from .autograd import LmmseFn


@dataclass
class FitState:
    log_tau: float
    log_sigma2: float
    step: int = 0
    seed: int = 0
    adam: dict = field(default_factory=dict)
    history: list = field(default_factory=list)

    def save(self, path: str):
        with open(path, "w") as f:
            json.dump(asdict(self), f)

    @staticmethod
    def load(path: str) -> "FitState":
        with open(path) as f:
            return FitState(**json.load(f))


def fit_design(plan, batch_fn, steps: int = 200, lr: float = 0.05, tau0: float = 8.0,
               sigma2_0: float = 1e-4, state: FitState | None = None, log_every: int = 0):
    """Adam on (log tau_rms, log sigma2) minimising mean |Hhat - H|^2.

    batch_fn(step) -> (h_ls, H): complex64 CUDA tensors [S, M, K, N] (LS
    estimates and true channels of a fresh batch).  Returns the FitState.
    """
    if state is None:
        state = FitState(log_tau=math.log(tau0), log_sigma2=math.log(sigma2_0))
    lt = torch.tensor(state.log_tau, dtype=torch.float64, requires_grad=True)
    ls = torch.tensor(state.log_sigma2, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([lt, ls], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    if state.adam:
        opt.load_state_dict({"state": {int(k): {kk: torch.tensor(vv, dtype=torch.float64)
                                                for kk, vv in v.items()}
                                       for k, v in state.adam["state"].items()},
                             "param_groups": state.adam["param_groups"]})
    for step in range(state.step, steps):
        h_ls, H = batch_fn(step)
        out = LmmseFn.apply(h_ls, torch.exp(lt), torch.exp(ls), plan)
        loss = (out - H).abs().pow(2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        state.step = step + 1
        state.history.append([float(loss.detach()), math.exp(lt.item()), math.exp(ls.item())])
        if log_every and (step % log_every == 0 or step + 1 == steps):
            print(f"fit step {step}: loss {state.history[-1][0]:.4e} tau {state.history[-1][1]:.3f} "
                  f"sigma2 {state.history[-1][2]:.3e}", flush=True)
    state.log_tau = lt.item()
    state.log_sigma2 = ls.item()
    sd = opt.state_dict()
    state.adam = {"state": {str(k): {kk: (vv.item() if torch.is_tensor(vv) else vv)
                                     for kk, vv in v.items()}
                            for k, v in sd["state"].items()},
                  "param_groups": sd["param_groups"]}
    return state
