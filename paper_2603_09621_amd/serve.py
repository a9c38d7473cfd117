"""Continuous-batching request loop over resident Gaussian sets.

Two kinds of request arrive over time:

* render: render a resident Gaussian set on a grid at a given scale of its LR box (rendering at
  an arbitrary resolution, §4.2);
* fit: a per-scan zero-shot fit (§3.3, Fig. 1) of ``steps`` Adam steps on a new scan.

The loop keeps every resident set on the device and admits queued requests in arrival order while
a batch slot is free and their HBM footprint fits the budget (workspace at the exact key count
times a headroom, output volume; for a fit also its parameters, moments and per-step buffers).  A
request larger than the whole budget still runs once nothing else is admitted.

Admitted renders are rendered together: one bin + forward launch sequence over up to 16 scans that
reads every set's own tensors (a forward-only workspace).  Requests that arrive while a render batch
is on the device join the next batch.  Admitted fits are packed into one batched fit whose scans
keep their own Adam step counters, so a fit that joins later simply starts at step 0 beside others
at later steps; each tick runs a chunk of batched steps.  Renders and fits run on two streams of
default priority, so their kernels overlap on the device.  Every result equals the result of the
same request run alone (the batched kernels are bitwise equal to the single-scan calls), which the
tests check.

Latency of a request = completion time (its batch's completion event observed by the loop) minus
its arrival time; the loop reports p50 / p99 per kind beside throughput.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import gs

# (offset in units of n, entries per Gaussian) of mu, log_scale, quat, amp, relax in the moment arrays
GROUP_SLICES = ((0, 3), (3, 3), (6, 4), (10, 1), (11, 1))
MAX_SCANS = 16
_SLACK = 64 << 10  # per-request allowance for section alignment in shared workspaces


@dataclass
class RenderRequest:
    set_id: int
    scale: float
    arrival: float = 0.0
    rid: int = -1
    grid: Optional[gs.Grid] = None
    footprint: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    result: Optional[torch.Tensor] = None
    error: Optional[str] = None

    kind = "render"

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class FitRequest:
    params: dict  # initial parameters (numpy, float32)
    lr_obs: np.ndarray  # [nz / zdown, ny, nx]
    dims: Tuple[int, int, int]  # HR grid (nx, ny, nz)
    steps: int = 100
    arrival: float = 0.0
    rid: int = -1
    footprint: int = 0
    keys: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    result: Optional[Dict[str, torch.Tensor]] = None
    loss: Optional[float] = None
    error: Optional[str] = None

    kind = "fit"

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class _Fit:
    """An admitted fit: its own parameter and moment tensors (valid while it is not packed)."""

    def __init__(self, req: FitRequest, device):
        self.req = req
        self.g = gs.Gaussians.from_numpy(req.params, device=device)
        if self.g.relax is None:
            self.g.relax = torch.ones_like(self.g.amp)
        self.n = self.g.n
        self.grid = gs.Grid(*req.dims)
        self.m = torch.zeros(12 * self.n, dtype=torch.float32, device=device)
        self.v = torch.zeros(12 * self.n, dtype=torch.float32, device=device)
        self.step = torch.zeros(1, dtype=torch.int32, device=device)
        self.obs = torch.from_numpy(np.ascontiguousarray(req.lr_obs, dtype=np.float32)).to(device).reshape(-1)
        self.done = 0


class Server:
    def __init__(self, sets: Sequence[gs.Gaussians], lr_dims: Sequence[Tuple[int, int, int]], hbm_budget: int,
                 opts: Optional[gs.Opts] = None, fit_opts: Optional[gs.FitOpts] = None, max_batch: int = MAX_SCANS,
                 max_fits: int = MAX_SCANS, fit_chunk: int = 5, headroom: float = 1.25, fit_headroom: float = 1.5,
                 keep_results: bool = True, device="cuda"):
        if len(sets) != len(lr_dims):
            raise ValueError("one LR box per set expected")
        self.sets = list(sets)
        self.lr_dims = [tuple(int(x) for x in d) for d in lr_dims]
        self.budget = int(hbm_budget)
        o = opts or gs.Opts()
        self.ropts = o.with_(forward_only=True)
        self.fo = fit_opts or gs.FitOpts(None)
        self.max_batch = max(1, min(max_batch, MAX_SCANS))
        self.max_fits = max(1, min(max_fits, MAX_SCANS))
        self.fit_chunk = max(1, fit_chunk)
        self.headroom, self.fit_headroom = headroom, fit_headroom
        self.keep_results = keep_results
        self.device = torch.device(device)
        self._streams = None
        self.keys: Dict[Tuple[int, float], int] = {}
        self.used = 0
        self.peak_used = 0
        self.done: List = []

    @property
    def rstream(self):
        return self._stream(0)

    @property
    def fstream(self):
        return self._stream(1)

    def _stream(self, k):
        if self._streams is None:  # created on first use (streams of default priority)
            self._streams = (torch.cuda.Stream(device=self.device), torch.cuda.Stream(device=self.device))
        return self._streams[k]

    def admissible(self, r, busy: bool, renders_waiting: int, fits_active: int) -> bool:
        """Admission rule for the queue head: a free slot of its kind and room in the HBM budget;
        a request larger than the whole budget is admitted only when nothing else is admitted."""
        if r.kind == "render" and renders_waiting >= 4 * self.max_batch:
            return False
        if r.kind == "fit" and fits_active >= self.max_fits:
            return False
        return not busy or self.used + r.footprint <= self.budget

    # ---- sizing ---------------------------------------------------------------------------------

    def render_grid(self, set_id: int, scale: float) -> gs.Grid:
        return gs.Grid.at_scale(self.lr_dims[set_id], scale)

    def key_count(self, set_id: int, scale: float) -> int:
        """Exact key count of a render (one synchronising count pass, cached per set and scale)."""
        k = (set_id, float(scale))
        if k not in self.keys:
            grid = self.render_grid(set_id, scale)
            probe = gs.Bins(self.sets[set_id].n, grid, self.ropts, 0, device=self.device)
            self.keys[k] = gs.gs_bin_query(self.sets[set_id], grid, self.ropts, probe)
        return self.keys[k]

    def prepare(self, scales: Sequence[float]) -> None:
        """Count the keys of every resident set at every scale ahead of serving."""
        for s in range(len(self.sets)):
            for sc in scales:
                self.key_count(s, sc)

    def _render_cap(self, req: RenderRequest) -> int:
        return max(1024, int(math.ceil(self.key_count(req.set_id, req.scale) * self.headroom)))

    def render_footprint(self, req: RenderRequest) -> int:
        grid = req.grid or self.render_grid(req.set_id, req.scale)
        ws = gs.gs_workspace_size(self.sets[req.set_id].n, grid, self.ropts, self._render_cap(req))
        return ws + 4 * grid.size + _SLACK

    def prepare_fit(self, req: FitRequest) -> None:
        """Key count and HBM footprint of a fit request (one synchronising count pass).

        A fit holds, for its whole life, its own parameters and Adam moments (12 + 24 floats per
        Gaussian) and observation; while it runs, its share of the packed batch: a second copy of
        parameters and moments, its gradients (48 floats per Gaussian), observation, I and W (and
        dL/dI when the loss is not fused), the fit scratch, the binning workspace at its key count
        times the headroom, and the count pass's probe workspace taken when the batch is planned."""
        g = gs.Gaussians.from_numpy(req.params, device=self.device)
        grid = gs.Grid(*req.dims)
        probe = gs.Bins(g.n, grid, self.fo.opts, 0, device=self.device)
        req.keys = gs.gs_bin_query(g, grid, self.fo.opts, probe)
        cap = max(1024, int(math.ceil(req.keys * self.fit_headroom)))
        ws = gs.gs_workspace_size(g.n, grid, self.fo.opts, cap)
        own = 4 * 36 * g.n + 4 * req.lr_obs.size
        per_vox = 4 * (3 if self.fo.zdown != self.fo.opts.bz else 2)
        packed = 4 * 48 * g.n + 4 * req.lr_obs.size + per_vox * grid.size + gs.gs_fit_scratch_bytes(grid)
        req.footprint = own + packed + ws + probe.ws_bytes + _SLACK

    # ---- request loop ---------------------------------------------------------------------------

    def run(self, requests: Sequence, realtime: bool = True, clock: Callable[[], float] = time.perf_counter,
            on_done: Optional[Callable] = None, log: Optional[Callable[[str], None]] = None,
            log_every: float = 15.0) -> dict:
        """Serve the requests (sorted by arrival time, in seconds from the start).  With realtime
        False every request is queued at once (arrival times are then only the order).  log, if
        given, receives a progress line every log_every seconds."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for i, r in enumerate(reqs):
            if r.rid < 0:
                r.rid = i
            if r.kind == "render":
                r.grid = self.render_grid(r.set_id, r.scale)
                r.footprint = self.render_footprint(r)
            elif not r.footprint:
                self.prepare_fit(r)
        torch.cuda.synchronize(self.device)
        pending = deque(reqs)
        queue: deque = deque()
        admitted_renders: deque = deque()
        fits: List[_Fit] = []  # fits of the packed batch
        joining: List[_Fit] = []  # admitted fits that join at the next chunk
        rflight = None  # (event, requests, keep-alive tensors, status host buffer)
        fflight = None  # (event, steps host buffer, chunk)
        packed = None  # batched fit state of `fits`
        repack = False
        self.done = []
        t0 = clock()
        if not realtime:
            for r in pending:
                r.arrival = 0.0
            queue.extend(pending)
            pending.clear()

        def now():
            return clock() - t0

        next_log = log_every

        def finish(r):
            self.done.append(r)
            if on_done is not None:
                on_done(r)
            if not self.keep_results:
                r.result = None

        while pending or queue or admitted_renders or fits or joining or rflight or fflight:
            t = now()
            if log is not None and t >= next_log:
                log(f"{t:.0f}s: {len(self.done)} done, {len(queue)} queued, {len(pending)} not yet arrived")
                next_log += log_every
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            progressed = False

            # ---- retire finished work
            if rflight is not None and rflight[0].query():
                ev, batch_reqs, keep, st_host = rflight
                rflight = None
                overflow = int(st_host[2])  # DevStatus: int64 n_keys, int32 overflow, int32 nonfinite
                tdone = now()
                if overflow:
                    for r in batch_reqs:  # cannot happen at exact key counts; counted again, run again
                        self.keys.pop((r.set_id, float(r.scale)), None)
                        self.used -= r.footprint
                        r.footprint = self.render_footprint(r)
                        self.used += r.footprint
                    admitted_renders.extendleft(reversed(batch_reqs))
                else:
                    views = keep[1]
                    for r, v in zip(batch_reqs, views):
                        r.result = v
                        r.t_done = tdone
                        self.used -= r.footprint
                        finish(r)
                    views = v = None
                # the batch's workspace and volume go now, not when these names are next rebound
                del ev, batch_reqs, keep, st_host
                progressed = True
            if fflight is not None and fflight[0].query():
                ev, steps_host, chunk = fflight
                fflight = None
                tdone = now()
                steps = steps_host.numpy().astype(np.int64)
                finished = []
                for k, f in enumerate(fits):
                    if steps[k] < f.done + chunk:  # a step overflowed its key capacity: plan again
                        repack = True
                    f.done = int(steps[k])
                    if f.done >= f.req.steps:
                        finished.append(f)
                if finished:
                    self._unpack(fits, packed)
                    losses = packed["buf"].loss.detach().cpu().numpy()
                    for k, f in enumerate(fits):
                        if f in finished:
                            f.req.result = {k2: getattr(f.g, k2) for k2 in gs.GROUPS}
                            f.req.loss = float(losses[k])
                            f.req.t_done = tdone
                            self.used -= f.req.footprint
                            finish(f.req)
                    fits = [f for f in fits if f not in finished]
                    packed = None
                    finished = f = None  # the finished fits' own tensors go now
                progressed = True

            # ---- admit in arrival order while slots and memory allow
            while queue:
                r = queue[0]
                busy = bool(admitted_renders or fits or joining or rflight or fflight)
                if not self.admissible(r, busy, len(admitted_renders), len(fits) + len(joining)):
                    break
                queue.popleft()
                r.t_admit = now()
                self.used += r.footprint
                self.peak_used = max(self.peak_used, self.used)
                if r.kind == "render":
                    admitted_renders.append(r)
                else:
                    joining.append(_Fit(r, self.device))
                progressed = True

            # ---- launch a render batch
            if rflight is None and admitted_renders:
                batch_reqs = [admitted_renders.popleft() for _ in range(min(self.max_batch, len(admitted_renders)))]
                rflight = self._launch_renders(batch_reqs)
                progressed = True

            # ---- launch a chunk of batched fit steps
            if fflight is None and (fits or joining):
                if packed is None or repack or joining:
                    if packed is not None:
                        self._unpack(fits, packed)
                        packed = None  # released before the new batch is built: never two at once
                    fits = fits + joining
                    joining = []
                    packed = self._pack(fits)
                    repack = False
                chunk = min(self.fit_chunk, min(f.req.steps - f.done for f in fits))
                fflight = self._launch_fit_chunk(packed, chunk)
                progressed = True

            if not progressed:
                if pending and not (rflight or fflight):
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.002)))
                else:
                    time.sleep(0.0001)
        torch.cuda.synchronize(self.device)
        return self.report(now())

    # ---- renders ------------------------------------------------------------------------------

    def _launch_renders(self, reqs: List[RenderRequest]):
        sets = [self.sets[r.set_id] for r in reqs]
        batch = gs.Batch.of_sets(sets, [r.grid for r in reqs])
        cap = sum(self._render_cap(r) for r in reqs)
        self.rstream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.rstream):
            bins = gs.Bins(0, batch, self.ropts, cap, device=self.device)
            I = torch.empty(batch.v_offsets[-1], dtype=torch.float32, device=self.device)
            gs.gs_bin_batch(None, batch, self.ropts, bins, stream=self.rstream)
            gs.gs_render_fwd_batch(None, batch, self.ropts, bins, I, None, stream=self.rstream)
            st_host = torch.empty(4, dtype=torch.int32, pin_memory=True)
            st_host.copy_(bins.ws[:16].view(torch.int32), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.rstream)
        return ev, reqs, (bins, batch.split(I)), st_host

    # ---- fits ---------------------------------------------------------------------------------

    def _pack(self, fits: List[_Fit]) -> dict:
        # the fits' own tensors were initialised on the caller's stream
        self.fstream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.fstream):
            batch = gs.Batch([f.n for f in fits], [f.grid for f in fits])
            g = gs.concat([f.g for f in fits])
            st = gs.FitState(g, nscans=len(fits))
            off = batch.g_offsets
            ntot = g.n
            # slice by slice into the packed moments (no concatenated temporaries)
            for k, f in enumerate(fits):
                a, b = off[k], off[k + 1]
                for c, w in GROUP_SLICES:
                    st.m[c * ntot + w * a:c * ntot + w * b].copy_(f.m[c * f.n:(c + w) * f.n])
                    st.v[c * ntot + w * a:c * ntot + w * b].copy_(f.v[c * f.n:(c + w) * f.n])
                st.step[k:k + 1].copy_(f.step)
            obs = torch.cat([f.obs for f in fits])
            bins = gs.plan_bins_batch(g, batch, self.fo.opts, headroom=self.fit_headroom, stream=self.fstream)
            buf = gs.FitBuffers(g.n, batch, relax=True, device=self.device,
                                need_dL_dI=self.fo.zdown != self.fo.opts.bz)
        return {"batch": batch, "g": g, "st": st, "obs": obs, "bins": bins, "buf": buf}

    def _unpack(self, fits: List[_Fit], packed: dict) -> None:
        """Copy the packed state back into every fit's own tensors (on the fit stream)."""
        g, st = packed["g"], packed["st"]
        off = packed["batch"].g_offsets
        ntot = g.n
        with torch.cuda.stream(self.fstream):
            for k, f in enumerate(fits):
                a, b = off[k], off[k + 1]
                for name in gs.GROUPS:
                    getattr(f.g, name).copy_(getattr(g, name)[a:b])
                for c, w in GROUP_SLICES:
                    f.m[c * f.n:(c + w) * f.n].copy_(st.m[c * ntot + w * a:c * ntot + w * b])
                    f.v[c * f.n:(c + w) * f.n].copy_(st.v[c * ntot + w * a:c * ntot + w * b])
                f.step.copy_(st.step[k:k + 1])
        self.fstream.synchronize()

    def _launch_fit_chunk(self, packed: dict, chunk: int):
        fo = gs.FitOpts(None, opts=self.fo.opts, zdown=self.fo.zdown, adam=self.fo.adam)
        with torch.cuda.stream(self.fstream):
            for _ in range(chunk):
                gs.gs_fit_step_batch(packed["st"], packed["obs"], packed["batch"], fo, packed["bins"], packed["buf"],
                                     stream=self.fstream)
            steps_host = torch.empty(len(packed["batch"]), dtype=torch.int32, pin_memory=True)
            steps_host.copy_(packed["st"].step, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.fstream)
        return ev, steps_host, chunk

    # ---- report -------------------------------------------------------------------------------

    def report(self, wall: float) -> dict:
        out = {"completed": len(self.done), "wall_s": wall, "requests_per_s": len(self.done) / max(wall, 1e-9),
               "peak_hbm_bytes": self.peak_used, "budget_bytes": self.budget}
        def stats(lat):
            lat = np.asarray(lat)
            return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                    "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                    "max_ms": float(lat.max() * 1e3)}

        for kind in ("render", "fit"):
            lat = [r.latency for r in self.done if r.kind == kind]
            if lat:
                out[kind] = stats(lat)
        scales = sorted({r.scale for r in self.done if r.kind == "render"})
        if scales:
            out["render_by_scale"] = {f"{sc:g}": stats([r.latency for r in self.done if r.kind == "render"
                                                        and r.scale == sc]) for sc in scales}
        return out


def run_workload(duration: float = 120.0, rate: float = 50.0, budget_gib: float = 64.0, nsets: int = 32,
                 fit_pool: int = 4, fit_steps: int = 100, seed: int = 5, device="cuda", log=None) -> dict:
    """The request-loop workload: ``nsets`` resident sets (synth.serving_sets), Poisson arrivals
    (synth.serving_arrivals: 90% renders at scales 2, 2.5, 3, 4 of a set's LR box, 10% fits of
    ``fit_steps`` steps on scans of a pool), served in real time under an HBM budget."""
    from . import synth

    def say(*a):
        if log:
            log(" ".join(str(x) for x in a))

    t0 = time.perf_counter()
    sets_np = synth.serving_sets(seed, nsets)
    pool = synth.serving_fit_pool(seed + 1, fit_pool)
    arrivals = synth.serving_arrivals(seed, rate, duration, nsets, fit_pool=fit_pool)
    say(f"serving workload generated in {time.perf_counter() - t0:.1f}s: {len(arrivals)} requests")
    sets = [gs.Gaussians.from_numpy(p, device=device) for p, _ in sets_np]
    server = Server(sets, [d for _, d in sets_np], hbm_budget=int(budget_gib * (1 << 30)), keep_results=False,
                    device=device)
    server.prepare((2.0, 2.5, 3.0, 4.0))
    fit_fp = []
    for p, lr, d in pool:
        r = FitRequest(p, lr, d, steps=fit_steps)
        server.prepare_fit(r)
        fit_fp.append((r.footprint, r.keys))
    reqs = []
    for t, kind, a, b in arrivals:
        if kind == "render":
            reqs.append(RenderRequest(a, b, arrival=t))
        else:
            p, lr, d = pool[a]
            reqs.append(FitRequest(p, lr, d, steps=fit_steps, arrival=t, footprint=fit_fp[a][0], keys=fit_fp[a][1]))
    torch.cuda.synchronize()
    say(f"serving {len(reqs)} requests over {duration:.0f}s")
    rep = server.run(reqs, realtime=True, log=log)
    rep["workload"] = (f"{nsets} resident sets ({sum(s.n for s in sets)} Gaussians), Poisson arrivals at {rate:g}/s "
                       f"for {duration:g}s: 90% renders at scales 2, 2.5, 3, 4; 10% fits of {fit_steps} steps "
                       f"(scans of <= 200k Gaussians); HBM budget {budget_gib:g} GiB")
    rep["offered"] = len(reqs)
    return rep


def main():
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="request loop over resident Gaussian sets")
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--sets", type=int, default=32)
    ap.add_argument("--fit-steps", type=int, default=100)
    ap.add_argument("--seed", type=int, default=5)
    a = ap.parse_args()
    rep = run_workload(a.duration, a.rate, a.budget_gib, a.sets, fit_steps=a.fit_steps, seed=a.seed,
                       log=lambda m: print("[serve]", m, file=sys.stderr, flush=True))
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
