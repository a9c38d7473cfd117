"""Fit steps captured in a HIP graph.

A fit step is about a dozen kernel launches (binning, forward, backward with the fused loss,
reduction with Adam).  ``FitGraph`` records ``steps`` consecutive steps of a (batched) fit once and
replays them with a single launch, removing the per-launch host work.  Everything a step touches
(parameters, moments, step counters, observations, workspace and buffers) is fixed at capture and
must stay allocated; the library's launches under capture hold no memsets, host synchronisations or
allocations.  A replay computes exactly what the same eager calls would (the tests check it bitwise).
"""
from __future__ import annotations

import torch

from . import gs


class FitGraph:
    def __init__(self, st: gs.FitState, lr_obs: torch.Tensor, batch: gs.Batch, fo: gs.FitOpts, bins: gs.Bins,
                 buf: gs.FitBuffers, steps: int = 1):
        if steps < 1:
            raise ValueError("steps must be >= 1")
        self.args = (st, lr_obs, batch, fo, bins, buf)
        self.steps = steps
        self.graph = torch.cuda.CUDAGraph()
        # the capture stream must not wait on work it cannot see: start from an idle device
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            for _ in range(steps):
                gs.gs_fit_step_batch(*self.args)
        torch.cuda.synchronize()

    def replay(self) -> None:
        """Run the captured steps on the current stream."""
        self.graph.replay()
