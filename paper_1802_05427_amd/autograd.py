"""torch.autograd.Function over the C ABI: the fixed-design block filter as a
differentiable function of the LS estimates and of the design parameters.

    h_hat = LmmseFn.apply(h_ls, tau_rms, sigma2, plan)

h_ls is a complex64 CUDA tensor [S, M, K, N]; tau_rms and sigma2 are float64
scalar tensors.  The forward (re)designs the plan's filters for (tau_rms,
sigma2) and filters h_ls; the backward calls lmmse_backward, which returns
dL/dh_ls = sum_b W_b^H G_b and the FP64 gradients of the design parameters
(implicit differentiation of the block solve).  Complex gradients follow
PyTorch's convention, dL/dRe + j dL/dIm, which is also the library's.
"""
from __future__ import annotations

import torch


class LmmseFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h_ls, tau_rms, sigma2, plan):
        tau = float(tau_rms)
        sig = float(sigma2)
        plan.set_design(tau, sig)
        out = plan.apply(h_ls)
        ctx.save_for_backward(h_ls)
        ctx.plan = plan
        ctx.design = (tau, sig)
        return out

    @staticmethod
    def backward(ctx, g):
        (h_ls,) = ctx.saved_tensors
        plan = ctx.plan
        tau, sig = ctx.design
        # the plan may have been redesigned since this forward
        plan.set_design(tau, sig)
        want = bool(ctx.needs_input_grad[1] or ctx.needs_input_grad[2])
        d_hls, d_tau, d_sig = plan.backward(h_ls, g.contiguous(), want_params=want)
        gt = torch.tensor(d_tau, dtype=torch.float64) if ctx.needs_input_grad[1] else None
        gs = torch.tensor(d_sig, dtype=torch.float64) if ctx.needs_input_grad[2] else None
        return (d_hls if ctx.needs_input_grad[0] else None), gt, gs, None


class SampleLmmseFn(torch.autograd.Function):
    """The sample-covariance estimator as a function of the LS estimates and
    the noise variance: each (slot, user, window) designs its filter from the
    window's own covariance over the antennas, so the gradient to h_ls runs
    through R as well as through the filtering.

        h_hat = SampleLmmseFn.apply(h_ls, sigma2, plan[, keep])

    keep=True keeps each window's FP64 design from the forward for the
    backward (lmmse_estimate_ls_keep / lmmse_backward_kept: 1.05 MB per
    198-wide window, released after the backward) where the plan allows it,
    instead of forming it again; autograd's check of the saved h_ls ties the
    backward to the forward's LS values.
    """

    @staticmethod
    def forward(ctx, h_ls, sigma2, plan, keep=False):
        sig = float(sigma2)
        nbytes = plan.design_state_bytes(int(h_ls.shape[0])) if keep else 0
        ctx.state = torch.empty(nbytes, dtype=torch.uint8, device=h_ls.device) if nbytes else None
        out = plan.estimate_ls(h_ls, sig, keep=ctx.state)
        ctx.save_for_backward(h_ls)
        ctx.plan = plan
        ctx.sigma2 = sig
        return out

    @staticmethod
    def backward(ctx, g):
        (h_ls,) = ctx.saved_tensors
        plan = ctx.plan
        plan.set_design(float("nan"), ctx.sigma2)
        want = bool(ctx.needs_input_grad[1])
        if ctx.state is not None:
            par = torch.empty(2, dtype=torch.float64, device=h_ls.device)
            d_hls, _, d_sig_t = plan.backward(h_ls, g.contiguous(), params_out=par, kept=ctx.state)
            ctx.state = None
            gs = d_sig_t.cpu() if want else None
        else:
            d_hls, _, d_sig = plan.backward(h_ls, g.contiguous(), want_params=want)
            gs = torch.tensor(d_sig, dtype=torch.float64) if want else None
        return (d_hls if ctx.needs_input_grad[0] else None), gs, None, None


def lmmse_filter(h_ls, tau_rms, sigma2, plan):
    """Functional form of LmmseFn."""
    return LmmseFn.apply(h_ls, tau_rms, sigma2, plan)
