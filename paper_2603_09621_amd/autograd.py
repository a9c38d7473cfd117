"""torch.autograd.Function over the rasterizer's forward and backward kernels.

``render(mu, log_scale, quat, amp, relax, grid)`` returns the rendered volume I [nz, ny, nx] as a
differentiable function of the five parameter tensors (§3.2 Eq. (rendering)); its backward calls
the library's hand-written gradient kernels (§3.3 gradient equations: brick-local partial sums,
a fixed-order per-Gaussian reduction, no atomics).  The binning workspace built in the forward is
kept for the backward, so the parameters must not be modified in place in between (torch's saved-
tensor version check enforces this).
"""
from __future__ import annotations

from typing import Optional

import torch

from . import gs


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, log_scale, quat, amp, relax, grid: gs.Grid, opts: gs.Opts, headroom: float):
        g = gs.Gaussians(mu.detach().contiguous(), log_scale.detach().contiguous(), quat.detach().contiguous(),
                         amp.detach().contiguous(), None if relax is None else relax.detach().contiguous())
        bins = gs.plan_bins(g, grid, opts, headroom=headroom)
        I, W, _ = gs.render(g, grid, opts, bins)
        gs.gs_status(bins)
        ctx.save_for_backward(g.mu, g.log_scale, g.quat, g.amp, *(() if g.relax is None else (g.relax,)), I, W)
        ctx.has_relax = g.relax is not None
        ctx.bins, ctx.grid, ctx.opts = bins, grid, opts
        ctx.mark_non_differentiable(W)
        return I, W

    @staticmethod
    def backward(ctx, dI, dW):  # dW: W is returned for inspection only
        saved = ctx.saved_tensors
        if ctx.has_relax:
            mu, ls, q, amp, relax, I, W = saved
        else:
            mu, ls, q, amp, I, W = saved
            relax = None
        g = gs.Gaussians(mu, ls, q, amp, relax)
        grads = gs.backward(g, ctx.grid, ctx.opts, ctx.bins, I, W, dI.contiguous().to(torch.float32))
        return grads.mu, grads.log_scale, grads.quat, grads.amp, grads.relax, None, None, None


def render(mu: torch.Tensor, log_scale: torch.Tensor, quat: torch.Tensor, amp: torch.Tensor,
           relax: Optional[torch.Tensor], grid: gs.Grid, opts: Optional[gs.Opts] = None, headroom: float = 1.25,
           return_weights: bool = False):
    """Differentiable render: I (and W if ``return_weights``) on ``grid``."""
    I, W = _Render.apply(mu, log_scale, quat, amp, relax, grid, opts or gs.Opts(), headroom)
    return (I, W) if return_weights else I
