"""The hard-coded gradient as a torch.autograd.Function adjoint.

Forward runs one HG evaluation (forward sweep, then the backward sweep that
rebuilds the states and carries the co-state; Sec. III.C) and keeps the
gradient it produced; backward scales that gradient by the incoming
cotangent.  No second sweep and no autograd graph through the propagation:
the memory is that of HG (Table I), independent of N.
"""
from __future__ import annotations

from typing import Optional

import torch

from .api import Problem, evaluate


class HGCost(torch.autograd.Function):
    """cost = HGCost.apply(u, problem, psi0, targets, dt, options)

    u: float64 device tensor (K, N) or (B, K, N); returns the cost(s) with
    shape () or (B,).  `options` is a dict of keyword arguments of
    paper_2304_06200_amd.evaluate (w_fid, w_pen, tau, dtype, renorm_every,
    schedule, mode, ckpt_every)."""

    @staticmethod
    def forward(ctx, u, problem: Problem, psi0, targets, dt: float, options: Optional[dict] = None):
        opts = dict(options or {})
        res = evaluate(problem, u.detach(), psi0, targets, dt, **opts)
        grad = res.grad if res.grad is not None else torch.zeros(
            (1,) + tuple(u.shape[-2:]), dtype=torch.float64, device=u.device)
        ctx.batched = u.dim() == 3
        ctx.save_for_backward(grad)
        cost = torch.as_tensor(res.cost, dtype=u.dtype, device=u.device)
        return cost if ctx.batched else cost[0]

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        if ctx.batched:
            gu = grad_out.reshape(-1, 1, 1) * g
        else:
            gu = grad_out * g[0]
        return gu, None, None, None, None, None


def hg_cost(problem: Problem, u, psi0, targets, dt: float, **options):
    """Differentiable cost of the amplitudes `u` (see HGCost)."""
    return HGCost.apply(u, problem, psi0, targets, dt, options)
