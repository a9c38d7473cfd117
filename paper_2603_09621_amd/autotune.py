"""Autotuner of the rasterizer's speed knobs.

The knobs change speed, not the method: the brick width along x (4, 8 or 16 voxels, 8 x 4 in y x z;
§3.3 uses 8 x 8 x 4), which changes results only by FP32 summation order, and three choices that
leave every result bitwise the same: the number of consecutive bricks whose keys one backward
workgroup orders together (8 with eight waves, or 2 or 1 with one wave), the size of the
backward's ordering window (the default or half of it) and the emit's LDS stage (4096 or 6144 keys per
workgroup, or chosen from the key capacity).  Which setting is fastest depends on the Gaussians'
extent relative to the brick, on the key counts and on how long-tailed they are, so the tuner
measures: it runs a few fit steps (or renders) of the caller's own workload, on copies of the
parameters, timed with HIP events on the launch stream, and searches the knobs one at a time
(coordinate descent: brick width first, then the others at the best width).  Choices are cached per
workload signature (grid sizes, Gaussian count and mean extent, bucketed) in memory and, if a path
is given, in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Optional, Sequence

import torch

from . import gs

CANDIDATES = (4, 8, 16)
# the result-invariant knobs, searched after the brick width, with their default first
KNOBS = (("bwd_bricks", (8, 2, 1)), ("bwd_window", (512, 256)), ("emit_stage", (0, 4096, 6144)))
FIT_KNOBS = ("bwd_bricks", "bwd_window", "emit_stage")
RENDER_KNOBS = ("emit_stage",)


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


def _key(o: gs.Opts) -> str:
    return f"bx{o.bx}/g{o.bwd_bricks}/w{o.bwd_window}/e{o.emit_stage}"


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

    def _search(self, key: str, base: gs.Opts, knobs: Sequence[str], measure: Callable[[gs.Opts], float]) -> gs.Opts:
        """Coordinate descent over brick width, then each knob in turn; cached under key."""
        if key not in self.cache:
            times: Dict[str, float] = {}

            def t(o: gs.Opts) -> float:
                k = _key(o)
                if k not in times:
                    times[k] = measure(o)
                return times[k]

            best = min((base.with_(bx=bx) for bx in self.candidates), key=t)
            for name, values in KNOBS:
                if name in knobs:
                    best = min((best.with_(**{name: v}) for v in values), key=t)
            self.cache[key] = {"opts": best.tuning, "ms": {k: round(v, 4) for k, v in sorted(times.items())}}
            self._save()
        entry = self.cache[key]
        tune = entry.get("opts", {"bx": entry.get("bx", 8)})  # older cache files hold the width only
        return base.with_(**tune)

    def fit_opts(self, g: gs.Gaussians, batch: gs.Batch, lr_obs: torch.Tensor, zdown: int = 4,
                 base: Optional[gs.Opts] = None, steps: int = 3, warmup: int = 1, headroom: float = 1.5) -> gs.Opts:
        """Fastest options for fit steps of (g, batch, lr_obs); g is not modified."""
        base = base or gs.Opts()

        def measure(opts: gs.Opts) -> float:
            gc = gs.Gaussians(*(None if x is None else x.clone() for x in (g.mu, g.log_scale, g.quat, g.amp, g.relax)))
            bins = gs.plan_bins_batch(gc, batch, opts, headroom=headroom)
            st = gs.FitState(gc, nscans=len(batch))
            buf = gs.FitBuffers(gc.n, batch, relax=gc.relax is not None, device=gc.amp.device,
                                need_dL_dI=zdown != opts.bz)
            fo = gs.FitOpts(None, opts=opts, zdown=zdown)
            ms = self._time(lambda: gs.gs_fit_step_batch(st, lr_obs, batch, fo, bins, buf), steps, warmup)
            gs.gs_status(bins)
            return ms

        return self._search(signature("fit", batch.grids, g, zdown), base, FIT_KNOBS, measure)

    def render_opts(self, g: gs.Gaussians, batch: gs.Batch, base: Optional[gs.Opts] = None, steps: int = 3,
                    warmup: int = 1, headroom: float = 1.25) -> gs.Opts:
        """Fastest options for bin + forward renders of (g, batch)."""
        base = base or gs.Opts()
        dev = g.amp.device if g.n else "cuda"
        I = torch.empty(batch.v_offsets[-1], dtype=torch.float32, device=dev)

        def measure(opts: gs.Opts) -> float:
            bins = gs.plan_bins_batch(g, batch, opts, headroom=headroom)

            def run():
                gs.gs_bin_batch(g, batch, opts, bins)
                gs.gs_render_fwd_batch(g, batch, opts, bins, I, None)

            ms = self._time(run, steps, warmup)
            gs.gs_status(bins)
            return ms

        return self._search(signature("render", batch.grids, g), base, RENDER_KNOBS, measure)
