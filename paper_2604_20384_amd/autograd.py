"""The Hilbert-Schmidt cost as a differentiable PyTorch function of the gates.

`hs_cost(G, problem)` returns C(G) = 1 - (1/N_s) sum_s |phi_s^dag G psi_s|^2 (Eq. costHS) as a
float64 tensor.  Its forward runs the library's forward sweep, which keeps layer checkpoints
in the problem's workspace (the problem's `ckpt_every` sets how many); its backward is the
library's adjoint sweep (Alg. 1's backward pass with the environments of Eq. environment),
recomputing each segment from its checkpoint.  The returned gradient is grad_out * grad C in
the complex-gradient convention of App. A (grad f = df/dx + i df/dy), which is also the
convention of PyTorch's complex `.grad`.

A problem holds the checkpoints of one forward sweep at a time: if it was used for anything
else between this function's forward and backward, the backward re-runs the forward sweep
first (same result, bitwise).

Both directions use the library's device-pointer calls: G, the cost and the gradient stay on the
device (on the problem's stream), with no host copy of the gates.
"""
from __future__ import annotations

import torch

from .api import Problem


class HSCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, G: torch.Tensor, problem: Problem):
        if not torch.is_complex(G):
            raise TypeError("G must be a complex tensor of shape (K, 4, 4)")
        Gd = G.detach().to(torch.device(f"cuda:{problem.device}"), torch.complex128).contiguous()
        cost, _ = problem.forward_dev(Gd)
        ctx.problem, ctx.Gd, ctx.epoch = problem, Gd, problem.epoch
        ctx.out_device, ctx.out_dtype = G.device, G.dtype
        return cost.clone().to(G.device)

    @staticmethod
    def backward(ctx, grad_out):
        p = ctx.problem
        if p.epoch != ctx.epoch:
            p.forward_dev(ctx.Gd)                 # the checkpoints were replaced: sweep again
        g = p.backward_dev()
        gt = g.to(ctx.out_device, ctx.out_dtype)
        return grad_out.to(gt.real.dtype) * gt, None


def hs_cost(G: torch.Tensor, problem: Problem) -> torch.Tensor:
    """Differentiable C(G) for a `Problem` (see module docstring)."""
    return HSCost.apply(G, problem)
