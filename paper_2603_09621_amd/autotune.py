"""Brick-width autotuner.

The brick partition of §3.3 (8 x 8 x 4 in the paper) is a speed knob: the library runs bricks of
4, 8 or 16 voxels along x (8 x 4 in y x z) with results equal up to FP32 summation order.  Which
width is fastest depends on the Gaussians' extent relative to the brick and on the key count, so
the tuner measures: it runs a few fit steps (or renders) of the caller's own workload at every
width, on copies of the parameters, times them with HIP events on the launch stream and keeps the
fastest.  Choices are cached per workload signature (grid sizes, Gaussian count and mean extent,
bucketed) in memory and, if a path is given, in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence

import torch

from . import gs

CANDIDATES = (4, 8, 16)


def _bucket(x: float, per_octave: int = 2) -> int:
    return int(round(per_octave * math.log2(max(x, 1.0))))


def signature(kind: str, grids: Sequence[gs.Grid], g: gs.Gaussians, zdown: int = 0) -> str:
    """Workload key: kind, scan count, total voxels and Gaussians (half-octave buckets), mean
    log-scale of the Gaussians relative to the mean voxel spacing (0.25 buckets) and zdown."""
    vox = sum(gr.size for gr in grids)
    if g.n:
        h = sum(sum(gr.spacing) / 3.0 * gr.size for gr in grids) / max(vox, 1)
        ext = float(g.log_scale.float().mean().item()) - math.log(h)
    else:
        ext = 0.0
    return f"{kind}|s{len(grids)}|v{_bucket(vox)}|n{_bucket(g.n + 1)}|e{round(4 * ext)}|z{zdown}"


class Tuner:
    def __init__(self, path: Optional[str] = None, candidates: Sequence[int] = CANDIDATES):
        self.path = path
        self.candidates = tuple(bx for bx in candidates if gs.brick_supported(bx, 8, 4))
        self.cache: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def _save(self):
        if not self.path:
            return
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    @staticmethod
    def _time(fn, steps: int, warmup: int) -> float:
        for _ in range(warmup):
            fn()
        s = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(steps):
            fn()
        b.record(s)
        b.synchronize()
        return a.elapsed_time(b) / steps

    def fit_opts(self, g: gs.Gaussians, batch: gs.Batch, lr_obs: torch.Tensor, zdown: int = 4,
                 base: Optional[gs.Opts] = None, steps: int = 3, warmup: int = 1, headroom: float = 1.5) -> gs.Opts:
        """Fastest brick width for fit steps of (g, batch, lr_obs); g is not modified."""
        base = base or gs.Opts()
        key = signature("fit", batch.grids, g, zdown)
        if key not in self.cache:
            times = {}
            for bx in self.candidates:
                opts = gs.Opts(bx=bx, by=base.by, bz=base.bz, cutoff=base.cutoff, eps=base.eps)
                gc = gs.Gaussians(*(None if t is None else t.clone() for t in
                                    (g.mu, g.log_scale, g.quat, g.amp, g.relax)))
                bins = gs.plan_bins_batch(gc, batch, opts, headroom=headroom)
                st = gs.FitState(gc, nscans=len(batch))
                buf = gs.FitBuffers(gc.n, batch, relax=gc.relax is not None, device=gc.amp.device,
                                    need_dL_dI=zdown != opts.bz)
                fo = gs.FitOpts(None, opts=opts, zdown=zdown)
                times[bx] = self._time(lambda: gs.gs_fit_step_batch(st, lr_obs, batch, fo, bins, buf), steps, warmup)
                gs.gs_status(bins)
                del gc, bins, st, buf
            best = min(times, key=times.get)
            self.cache[key] = {"bx": best, "ms": {str(k): round(v, 4) for k, v in times.items()}}
            self._save()
        bx = int(self.cache[key]["bx"])
        return gs.Opts(bx=bx, by=base.by, bz=base.bz, cutoff=base.cutoff, eps=base.eps)

    def render_opts(self, g: gs.Gaussians, batch: gs.Batch, base: Optional[gs.Opts] = None, steps: int = 3,
                    warmup: int = 1, headroom: float = 1.25) -> gs.Opts:
        """Fastest brick width for bin + forward renders of (g, batch)."""
        base = base or gs.Opts()
        key = signature("render", batch.grids, g)
        if key not in self.cache:
            times = {}
            dev = g.amp.device if g.n else "cuda"
            nv = batch.v_offsets[-1]
            I = torch.empty(nv, dtype=torch.float32, device=dev)
            for bx in self.candidates:
                opts = gs.Opts(bx=bx, by=base.by, bz=base.bz, cutoff=base.cutoff, eps=base.eps)
                bins = gs.plan_bins_batch(g, batch, opts, headroom=headroom)

                def run():
                    gs.gs_bin_batch(g, batch, opts, bins)
                    gs.gs_render_fwd_batch(g, batch, opts, bins, I, None)

                times[bx] = self._time(run, steps, warmup)
                gs.gs_status(bins)
                del bins
            best = min(times, key=times.get)
            self.cache[key] = {"bx": best, "ms": {str(k): round(v, 4) for k, v in times.items()}}
            self._save()
        bx = int(self.cache[key]["bx"])
        return gs.Opts(bx=bx, by=base.by, bz=base.bz, cutoff=base.cutoff, eps=base.eps)
