"""torch.autograd.Function over the C ABI: forward = ph_forward_batch,
backward = ph_backward_batch (the hand-written adjoint sweep).

The differentiable input is the float32 tensor [sum m, 7] of log10
parameters {alpha, beta, delta, eps, zeta, lam_match, lam_mismatch} of every
read base; the output is float64 log10 L of every pair in output order.
Torch supplies device memory, the current stream and the autograd graph;
all arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import torch

from . import binding


class PairHMMLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log10_params: torch.Tensor, plan: "binding.Plan", dev: "binding.DeviceProblem"):
        lp = log10_params.detach().contiguous()
        assert lp.dtype == torch.float32 and lp.is_cuda and lp.shape[1] == 7
        out, status = plan.forward(dev, lp)
        ctx.plan, ctx.dev = plan, dev
        ctx.save_for_backward(lp)
        ctx.mark_non_differentiable(status)
        return out.clone(), status.clone()

    @staticmethod
    def backward(ctx, grad_out, grad_status):
        (lp,) = ctx.saved_tensors
        g = grad_out.to(torch.float64).contiguous()
        grad = ctx.plan.backward(ctx.dev, g, log10_params=lp)
        return grad.clone(), None, None


def pairhmm_log10_likelihood(log10_params, plan, dev):
    """log10 L of every pair; differentiable w.r.t. log10_params."""
    out, _ = PairHMMLogLik.apply(log10_params, plan, dev)
    return out
