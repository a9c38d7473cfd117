"""Benchmark of the rasterizer's hot path on one MI355X.

A step is one iteration of the per-scan zero-shot fit (gs_fit_step): bin (prep, key generation,
radix sort, brick offsets) -> forward render -> z-mean-of-4 L1 loss -> backward (brick partials,
reduction, chain rule) -> Adam.  Workload: HR 256x256x128 phantom (60 soft ellipsoids, N(0, 0.01^2)
noise), LR observation = mean of 4 consecutive z slices, 500k Gaussians initialised on the LR
lattice.  Inputs are resident in HBM before timing starts.

Metric: Gaussian-voxel evaluations per second (forward + backward): the number of useful pairs
(voxel, Gaussian with d^2 <= 9) of every timed step's render, summed, over the timed wall time.
Each useful pair is evaluated once in the forward and once in the backward.  The pair count comes
from replaying the same steps from a snapshot (the kernels are deterministic) with a counting pass
after each step.

Prints one JSON line.  --gpus N with N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per useful pair (voxel, Gaussian with d^2 <= 9), per-Gaussian constants hoisted
# (the exponent's matrix pre-scaled, log2 r folded in):
#  flops: forward 21 (delta, the quadratic form, exp2 and the two accumulations), backward 50 (delta,
#  P delta, d^2, exp2, t, dA, kappa, dmu, the six second moments, dr);
#  issue slots: forward 20, backward 38 (VALU instructions with exp2 charged 4 slots as a quarter-rate
#  transcendental; compares and selects count).
F_FWD, F_BWD = 21, 50
C_FWD, C_BWD = 20, 38
# MI355X published FP32 vector peak (packed FMA: 256 CU x 64 lanes x 4 flops x 2.4 GHz).
FP32_PEAK_TFLOPS = 157.3
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: FP32 VALU lane-instructions per second (non-packed issue).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def alu_roofline(name, ms, pairs, flops_per_pair, slots_per_pair, traffic=None):
    """Flops per launch over the launch's mean duration against the FP32 vector peak, and the same
    launch as issue slots against the non-packed VALU issue rate."""
    tflops = pairs * flops_per_pair / (ms * 1e-3) / 1e12
    tslots = pairs * slots_per_pair / (ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": name, "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
            "flops_per_pair": flops_per_pair, "ms": round(ms, 5),
            "issue": {"achieved": round(tslots, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tlane-instr/s",
                      "frac": round(tslots / VALU_PEAK_TOPS, 4), "slots_per_pair": slots_per_pair}}


def hbm_fractions(kern, K, N, passes):
    """Algorithmic HBM bytes per launch of the binning, reduction and Adam kernels (what each must
    read and write once) over the launch's mean duration, against 8 TB/s."""
    per_launch = {
        # parameters 13 floats read; evaluation (48 B) + culling (32 B) records, key count, run cache
        "prep_count": 52 * N + (48 + 32 + 4 + 32) * N,
        # run cache + key offsets read; (brick id, Gaussian id) per key written
        "emit": (32 + 4) * N + 8 * K,
        # one digit histogram pass: brick ids read
        "radix_hist": 4 * K,
        # a scatter pass: brick ids and slots read and written; the last pass writes the Gaussian id
        # (read by slot) instead of the brick id, i.e. 4 B more per key in one of the passes (the
        # brick list bounds it also writes are 8 B per brick)
        "radix_scatter": 16 * K + 4 * K / passes,
        # partials 48 B per key and key offsets read; 12 parameters, m, v read and written, the
        # 12 gradients written
        "reduce_adam": 48 * K + 4 * N + 12 * 4 * (3 + 3 + 1) * N,
    }
    out = {}
    for k, b in per_launch.items():
        if k in kern:
            ms = kern[k]["avg_ms"]
            gbs = b / (ms * 1e-3) / 1e9
            out[k] = {"bytes": int(b), "ms": round(ms, 5), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dims", type=int, nargs=3, default=(256, 256, 128))
    ap.add_argument("--n", type=int, default=500000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--bx", type=int, default=8, help="brick width along x (4, 8 or 16)")
    ap.add_argument("--bwd-bricks", type=int, default=8,
                    help="bricks per backward workgroup (8: eight waves; 2 or 1: one wave)")
    ap.add_argument("--bwd-window", type=int, default=512,
                    help="backward ordering window: 512 (the default size) or 256 (half of it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle fit steps timed for the CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven-scan comparison")
    ap.add_argument("--no-graph", action="store_true", help="skip timing the fit step replayed from a HIP graph")
    ap.add_argument("--batch-steps", type=int, default=100, help="timed steps of the batched comparison")
    ap.add_argument("--serve-seconds", type=float, default=120.0,
                    help="seconds of Poisson arrivals for the request-loop section (0: skip)")
    ap.add_argument("--plain-reps", type=int, default=400,
                    help="timed graph replays of the plain 64x64x32 / 20k render + gradient (0: skip)")
    ap.add_argument("--no-cpu-aniso", action="store_true",
                    help="skip timing the oracle on the anisotropic 2M-Gaussian render + gradient")
    ap.add_argument("--aniso-steps", type=int, default=5,
                    help="timed render+gradient steps of the anisotropic 2M-Gaussian workload (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run one plain device-to-device copy of this many MiB (a known-size "
                         "kernel against which profiler byte counters are calibrated)")
    return ap.parse_args()


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from a committed counter summary
    (profiles/*_traffic.json), if it was taken on the current kernel source; else None."""
    import glob

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))):
        try:
            rec = json.load(open(path))
            if rec.get("kernel") != kernel or rec.get("workload_key") != workload:
                continue
            sha = hashlib.sha256(open(os.path.join(ROOT, rec["source"]), "rb").read()).hexdigest()
            if rec.get("source_sha256") == sha:
                return float(rec["hbm_bytes_per_launch"])
        except (OSError, ValueError, KeyError):
            continue
    return None


def batch_section(args, dev):
    """16 uneven single-scan fits: one batched step (all scans, one launch per phase, autotuned brick
    width, replayed from a HIP graph; then the same with eager launches) against the same 16 fits
    stepped one scan at a time through the plain single-scan call at the same brick width.  Both
    start from the same parameters and take the same number of steps; their final parameters must be
    bitwise equal."""
    import numpy as np
    import torch

    from paper_2603_09621_amd import autotune, graph, gs, synth

    t0 = time.time()
    scans = synth.workload_batch(seed=4)
    print(f"[bench] batch workload: {len(scans)} scans in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    grids = [gs.Grid(*d) for _, _, d in scans]
    sets = [gs.Gaussians.from_numpy(p, device=dev) for p, _, _ in scans]
    obs = [torch.from_numpy(lr).to(dev) for _, lr, _ in scans]
    batch = gs.Batch([x.n for x in sets], grids)
    g_all = gs.concat(sets)
    obs_all = torch.cat([o.reshape(-1) for o in obs])
    tuner = autotune.Tuner()
    opts = tuner.fit_opts(g_all, batch, obs_all, zdown=4, steps=2)
    tuned = next(iter(tuner.cache.values()))
    print(f"[bench] autotuned {opts.tuning}", file=sys.stderr, flush=True)
    fo = gs.FitOpts(None, opts=opts, zdown=4)
    stream = torch.cuda.current_stream()
    K, W = args.batch_steps, 2

    def timed(fn, k):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    # batched + graph
    bins = gs.plan_bins_batch(g_all, batch, opts, headroom=1.5)
    st = gs.FitState(g_all, nscans=len(batch))
    buf = gs.FitBuffers(g_all.n, batch, relax=g_all.relax is not None, device=dev, need_dL_dI=False)
    for _ in range(W):
        gs.gs_fit_step_batch(st, obs_all, batch, fo, bins, buf)
    gs.gs_status(bins)
    fg = graph.FitGraph(st, obs_all, batch, fo, bins, buf, steps=1)
    ms_batched = timed(fg.replay, K)
    gs.gs_status(bins)
    # K more batched steps with eager launches (the graph's gain)
    ms_eager = timed(lambda: gs.gs_fit_step_batch(st, obs_all, batch, fo, bins, buf), K)
    gs.gs_status(bins)
    # plain: every scan on its own, one after the other
    plain = []
    for x, gr, o in zip(sets, grids, obs):
        b1 = gs.plan_bins(x, gr, opts, headroom=1.5)
        plain.append((x, gs.FitState(x), o, gs.FitOpts(gr, opts=opts, zdown=4), b1,
                      gs.FitBuffers(x.n, gr, relax=x.relax is not None, device=dev)))
    for _ in range(W):
        for x, st1, o, fo1, b1, buf1 in plain:
            gs.gs_fit_step(st1, o, fo1, b1, buf1)

    def plain_round():
        for x, st1, o, fo1, b1, buf1 in plain:
            gs.gs_fit_step(st1, o, fo1, b1, buf1)

    ms_plain = timed(plain_round, K)
    # the plain path's time per scan (the catch-up steps below, timed scan by scan)
    per_scan = np.zeros(len(plain))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in plain]
    for _ in range(K):  # the plain fits catch up with the batched one (W + 2K steps each)
        for (x, st1, o, fo1, b1, buf1), (ea, eb) in zip(plain, evs):
            ea.record(stream)
            gs.gs_fit_step(st1, o, fo1, b1, buf1)
            eb.record(stream)
        torch.cuda.synchronize()
        per_scan += [ea.elapsed_time(eb) for ea, eb in evs]
    per_scan /= K
    for x, st1, o, fo1, b1, buf1 in plain:
        gs.gs_status(b1)
    off = batch.g_offsets
    equal = all(torch.equal(getattr(g_all, k)[off[j]:off[j + 1]], getattr(x, k))
                for j, x in enumerate(sets) for k in gs.GROUPS if getattr(x, k) is not None)
    dims = [list(d) for _, _, d in scans]
    return {
        "workload": f"{len(scans)} uneven single-scan fits (HR grids {min(d[0] for d in dims)}..{max(d[0] for d in dims)}"
                    f" in x/y, {min(d[2] for d in dims)}..{max(d[2] for d in dims)} in z; {g_all.n} Gaussians, "
                    f"{batch.v_offsets[-1]} HR voxels in total), z-mean-of-4 L1 + Adam",
        "brick": [opts.bx, opts.by, opts.bz],
        "tuning": opts.tuning,
        "tuner_ms_per_step": tuned["ms"],
        "steps": K,
        "ms_per_batched_step": ms_batched / K,
        "ms_per_plain_round": ms_plain / K,
        "scan_iters_per_s_batched": len(scans) * K / (ms_batched / 1e3),
        "scan_iters_per_s_plain": len(scans) * K / (ms_plain / 1e3),
        "speedup": ms_plain / ms_batched,
        "hip_graph": True,
        "bitwise_equal_to_plain": bool(equal),
        "ms_per_batched_step_eager": ms_eager / K,
        "plain_ms_per_scan": [{"dims": d, "n": x.n, "ms": round(float(t), 4)}
                              for d, x, t in sorted(zip(dims, sets, per_scan), key=lambda z: z[1].n)],
    }


def plain_section(args, dev):
    """The plain render + gradient (64x64x32, 20k Gaussians, MSE against a U(0,1) target): one
    repetition = bin, forward, MSE loss and dL/dI, backward with the reduction, captured once in a
    HIP graph and replayed; per-replay times from HIP events on the replay stream (median, p99), and
    the median of the same calls launched eagerly."""
    import numpy as np
    import torch

    from paper_2603_09621_amd import gs, synth

    p, T_np = synth.workload_plain(1, (64, 64, 32), 20000)
    grid = gs.Grid(64, 64, 32)
    opts = gs.Opts(bx=args.bx)
    g = gs.Gaussians.from_numpy(p, device=dev)
    T = torch.from_numpy(T_np).to(dev)
    bins = gs.plan_bins(g, grid, opts, headroom=1.25)
    I = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    W = torch.empty_like(I)
    gI = torch.empty_like(I)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    scratch = torch.empty(gs.gs_loss_scratch_bytes(I.numel()), dtype=torch.uint8, device=dev)
    grads = gs.Grads.empty(g.n, relax=g.relax is not None, device=dev)

    def step():
        gs.gs_bin(g, grid, opts, bins)
        gs.gs_render_fwd(g, grid, opts, bins, I, W)
        gs.gs_loss_mse(I, T, gI, loss, scratch)
        gs.gs_render_bwd(g, grid, opts, bins, I, W, gI, grads)

    for _ in range(5):
        step()
    gs.gs_status(bins)
    ref = grads.mu.clone()
    pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    gs.gs_count_pairs(g, grid, opts, bins, pairs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def per_rep(fn, reps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in ev])

    for _ in range(10):
        graph.replay()
    t_graph = per_rep(graph.replay, args.plain_reps)
    same = bool(torch.equal(grads.mu, ref))
    t_eager = per_rep(step, args.plain_reps)
    gs.gs_status(bins)
    U = int(pairs.item())
    med = float(np.median(t_graph))
    return {
        "workload": "plain render + gradient: 64x64x32, 20000 Gaussians (mu ~ U(volume), log-scale ~ N(ln 1.5, 0.3), "
                    "uniform rotations, A ~ U(0,1)), MSE vs U(0,1) target; bin + forward + loss + backward + reduction",
        "reps": args.plain_reps,
        "hip_graph": True,
        "ms_median": med,
        "ms_p99": float(np.percentile(t_graph, 99)),
        "ms_median_eager": float(np.median(t_eager)),
        "useful_pairs": U,
        "evals_per_s": U / (med * 1e-3),
        "replay_equals_eager": same,
    }


def aniso_section(args, dev):
    """Render + gradient of the anisotropic workload (320x320x256, 2M Gaussians, log-scale std 0.8,
    axis ratio <= 8, random rotations, MSE against a U(0,1) target): one step = bin, forward, MSE loss
    and dL/dI, backward with the reduction to per-Gaussian gradients (no optimiser step)."""
    import torch

    from paper_2603_09621_amd import gs, synth

    t0 = time.time()
    p, T_np = synth.workload_aniso()
    dims = (320, 320, 256)
    print(f"[bench] anisotropic workload in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    grid = gs.Grid(*dims)
    opts = gs.Opts(bx=args.bx, bwd_bricks=args.bwd_bricks, bwd_window=args.bwd_window)
    g = gs.Gaussians.from_numpy(p, device=dev)
    T = torch.from_numpy(T_np).to(dev)
    bins = gs.plan_bins(g, grid, opts, headroom=1.1)
    I = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    W = torch.empty_like(I)
    gI = torch.empty_like(I)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    scratch = torch.empty(gs.gs_loss_scratch_bytes(I.numel()), dtype=torch.uint8, device=dev)
    grads = gs.Grads.empty(g.n, relax=g.relax is not None, device=dev)

    def step():
        gs.gs_bin(g, grid, opts, bins)
        gs.gs_render_fwd(g, grid, opts, bins, I, W)
        gs.gs_loss_mse(I, T, gI, loss, scratch)
        gs.gs_render_bwd(g, grid, opts, bins, I, W, gI, grads)

    for _ in range(2):
        step()
    st = gs.gs_status(bins)
    pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    gs.gs_count_pairs(g, grid, opts, bins, pairs)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.aniso_steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.aniso_steps
    U = int(pairs.item())
    cpu = None
    if not args.no_cpu_aniso:
        import numpy as np

        import oracle

        del bins, I, W, gI, scratch, grads
        threads = oracle.default_threads()
        print(f"[bench] oracle anisotropic render + gradient on {threads} host threads", file=sys.stderr, flush=True)
        og = oracle.Grid(*dims)
        c0 = time.perf_counter()
        Io, Wo, _ = oracle.render(p, og, threads=threads)
        _, go = oracle.mse_loss(Io, T_np)
        oracle.grad(p, og, Io, Wo, go, threads=threads)
        cpu_s = time.perf_counter() - c0
        cpu = {"s_per_step": cpu_s, "cores": threads, "kind": "oracle", "evals_per_s": U / cpu_s,
               "sample": "one FP64 forward + MSE + gradient of the full workload"}
        del Io, Wo, go
    return {
        "workload": f"anisotropic render + gradient: HR {dims[0]}x{dims[1]}x{dims[2]}, {g.n} Gaussians (log-scale "
                    f"std 0.8, axis ratio <= 8, random rotations), MSE vs U(0,1) target; bin + forward + loss + "
                    f"backward + reduction per step",
        "brick": [opts.bx, opts.by, opts.bz],
        "steps": args.aniso_steps,
        "ms_per_step": ms,
        "keys": st["n_keys"],
        "useful_pairs": U,
        "evals_per_s": U / (ms * 1e-3),  # useful pairs per second, as the headline value
        "cpu_oracle": cpu,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_09621_amd import gs, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dims = tuple(args.dims)
    t0 = time.time()
    print(f"[bench] generating workload {dims} n={args.n}", file=sys.stderr, flush=True)
    p, lr_obs, _ = synth.workload_fit(args.seed, dims, args.n)
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    grid = gs.Grid(*dims)
    g = gs.Gaussians.from_numpy(p, device=dev)
    fo = gs.FitOpts(grid, opts=gs.Opts(bx=args.bx, bwd_bricks=args.bwd_bricks, bwd_window=args.bwd_window))
    obs = torch.from_numpy(lr_obs).to(dev)
    bins = gs.plan_bins(g, grid, fo.opts, headroom=1.5)
    st = gs.FitState(g)
    buf = gs.FitBuffers(g.n, grid, relax=g.relax is not None, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        gs.gs_fit_step(st, obs, fo, bins, buf)

    for _ in range(args.warmup):
        step()
    keys_warm = gs.gs_status(bins)["n_keys"]
    torch.cuda.synchronize()
    snap = {k: getattr(g, k).clone() for k in gs.GROUPS if getattr(g, k) is not None}
    snap_m, snap_v, snap_step = st.m.clone(), st.v.clone(), st.step.clone()

    # ---- timed region -------------------------------------------------------------------------
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)
    status = gs.gs_status(bins, raise_on_error=False)
    if status["rc"] != 0:
        print(f"[bench] status after timed steps: {status}", file=sys.stderr, flush=True)
        sys.exit(3)
    final = {k: getattr(g, k).clone() for k in snap}
    loss_end = float(buf.loss.item())

    # ---- replay: useful pairs per step + per-kernel durations (HIP events on the launch stream) ---
    for k, v in snap.items():
        getattr(g, k).copy_(v)
    st.m.copy_(snap_m)
    st.v.copy_(snap_v)
    st.step.copy_(snap_step)
    total_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    gs.profile_reset()
    gs.profile_enable(True)
    for _ in range(args.steps):
        step()
        gs.profile_enable(False)
        gs.gs_count_pairs(g, grid, fo.opts, bins, cnt)
        total_pairs += cnt
        gs.profile_enable(True)
    gs.profile_enable(False)
    prof = gs.profile_read()
    torch.cuda.synchronize()
    replay_same = all(torch.equal(getattr(g, k), final[k]) for k in final)
    U = int(total_pairs.item())
    t_step = gpu_ms / 1e3 / args.steps
    value = U / (gpu_ms / 1e3)

    kern = {name: {"launches": n, "avg_ms": tot / n} for name, (n, tot) in prof.items() if n}
    fwd_ms = kern.get("render_fwd", {}).get("avg_ms", float("nan"))
    bwd_ms = kern.get("render_bwd", {}).get("avg_ms", float("nan"))
    U_step = U / args.steps
    wl = f"fit {dims[0]}x{dims[1]}x{dims[2]} n={args.n} bx={args.bx}"
    kernel_roofline = {
        "render_fwd": alu_roofline("render_fwd", fwd_ms, U_step, F_FWD, C_FWD, traffic_from_profiles("render_fwd", wl)),
        "render_bwd": alu_roofline("render_bwd", bwd_ms, U_step, F_BWD, C_BWD, traffic_from_profiles("render_bwd", wl)),
    }
    dom = "render_bwd" if bwd_ms >= fwd_ms else "render_fwd"
    roofline = kernel_roofline[dom]

    # evaluation counts at the state after the timed steps: how much of the issued work is useful
    ev = torch.zeros(6, dtype=torch.int64, device=dev)
    gs.gs_count_evals(g, grid, fo.opts, bins, ev)
    ev = dict(zip(gs.EVAL_COUNTS, (int(x) for x in ev.cpu())))
    K_end = status["n_keys"]
    cull = {
        "keys": K_end,
        "useful_pairs": ev["useful_pairs"],
        "brick_candidates_per_useful": round(K_end * fo.opts.bx * 32 / max(ev["useful_pairs"], 1), 3),
        "fwd_evals_per_useful": round(ev["fwd_evals"] / max(ev["useful_pairs"], 1), 3),
        "fwd_issued_per_useful": round(ev["fwd_issued"] / max(ev["useful_pairs"], 1), 3),
        "bwd_evals_per_useful": round(ev["bwd_evals"] / max(ev["useful_pairs"], 1), 3),
        "bwd_issued_per_useful": round(ev["bwd_issued"] / max(ev["useful_pairs"], 1), 3),
        "bwd_box_rows_per_key": round(ev["bwd_box_rows"] / max(K_end, 1), 3),
        "fwd_slot_evals_per_s": ev["fwd_evals"] / (fwd_ms * 1e-3),
        "bwd_slot_evals_per_s": ev["bwd_evals"] / (bwd_ms * 1e-3),
    }
    nbricks = -(-dims[0] // fo.opts.bx) * -(-dims[1] // 8) * -(-dims[2] // 4)
    passes = max(1, -(-max(1, (nbricks - 1).bit_length()) // 8))
    hbm = hbm_fractions(kern, K_end, args.n, passes)
    # what a plain device-to-device copy reaches here (bytes read + written over its duration): the
    # practical ceiling of the HBM-bound kernels, beside the published 8 TB/s
    copy_src = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    copy_dst = torch.empty_like(copy_src)
    copy_dst.copy_(copy_src)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record()
    for _ in range(5):
        copy_dst.copy_(copy_src)
    ce1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * copy_src.numel() * 4 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del copy_src, copy_dst
    for v in hbm.values():
        v["frac_of_copy"] = round(v["GBps"] / copy_gbps, 4)
    hbm["device_copy_GBps"] = round(copy_gbps, 1)

    # the same steps replayed from a HIP graph (one captured fit step per replay)
    ms_graph = None
    if not args.no_graph:
        from paper_2603_09621_amd import graph

        fg = graph.FitGraph(st, obs, gs.Batch([g.n], [grid]), fo, bins, buf, steps=1)
        fg.replay()
        torch.cuda.synchronize()
        ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ga.record(stream)
        for _ in range(args.steps):
            fg.replay()
        gb.record(stream)
        torch.cuda.synchronize()
        ms_graph = ga.elapsed_time(gb) / args.steps
        if gs.gs_status(bins, raise_on_error=False)["rc"] != 0:
            ms_graph = None
        del fg

    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- CPU baseline: the oracle on the host cores, full fit steps of the same workload ---------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle.default_threads()
        print(f"[bench] oracle fit steps on {threads} host threads", file=sys.stderr, flush=True)
        og = oracle.Grid(*dims)
        lr = dict(zip(oracle.GROUPS, [float(np.float32(x)) for x in fo.adam.lr]))

        def oracle_steps(k, nthreads):
            """k fit steps from the workload's initial state; the time of each."""
            mom = {key: np.zeros(np.shape(p[key])) for key in oracle.GROUPS}
            vel = {key: np.zeros(np.shape(p[key])) for key in oracle.GROUPS}
            cur, times = p, []
            for s in range(k):
                c0 = time.perf_counter()
                _, newp, mom, vel, _ = oracle.fit_step(cur, lr_obs, og, mom, vel, s + 1, lr, threads=nthreads)
                times.append(time.perf_counter() - c0)
                cur = {key: np.asarray(v, np.float32) for key, v in newp.items()}
            return times

        pairs0 = oracle.count_pairs(p, og, threads=threads)
        times = oracle_steps(args.cpu_steps, threads)
        cpu_s = float(np.median(times))
        print("[bench] oracle fit step on 1 host thread", file=sys.stderr, flush=True)
        one_s = oracle_steps(1, 1)[0]
        cpu = {"value": pairs0 / cpu_s, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"median of {args.cpu_steps} FP64 fit steps (render, z-mean L1, gradient, Adam) of the full "
                         f"{dims[0]}x{dims[1]}x{dims[2]} / {args.n}-Gaussian workload from its initial state, "
                         f"{pairs0} useful pairs per step, {cpu_s:.2f} s per step on {threads} threads; "
                         f"one step on 1 thread {one_s:.2f} s",
               "s_per_step": cpu_s, "s_per_step_all": [round(x, 3) for x in times],
               "s_per_step_1core": one_s, "value_1core": pairs0 / one_s}

    plain = None
    if args.plain_reps > 0:
        print("[bench] plain 64x64x32 / 20k render + gradient", file=sys.stderr, flush=True)
        plain = plain_section(args, dev)

    aniso = None
    if args.aniso_steps > 0:
        del bins, st, buf, g
        torch.cuda.empty_cache()
        aniso = aniso_section(args, dev)
        torch.cuda.empty_cache()

    batched = None
    if not args.no_batch:
        del snap, final
        torch.cuda.empty_cache()
        batched = batch_section(args, dev)
    serving = None
    if args.serve_seconds > 0:
        from paper_2603_09621_amd import serve

        torch.cuda.empty_cache()
        serving = serve.run_workload(duration=args.serve_seconds,
                                     log=lambda m: print("[bench]", m, file=sys.stderr, flush=True))

    out = {
        "metric": "Gaussian\u2013voxel evals/s (fwd+bwd), fit iters/s vs plain; p50/p99 render latency",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"single-scan zero-shot fit: HR {dims[0]}x{dims[1]}x{dims[2]} phantom, LR = z-mean "
                               f"of 4, {args.n} Gaussians on the LR lattice, L1 + Adam",
                   "global_batch": 1, "brick": [fo.opts.bx, fo.opts.by, fo.opts.bz], "tuning": fo.opts.tuning},
        "fit_iters_per_s": 1.0 / t_step,
        "ms_per_step_hip_graph": ms_graph,
        "useful_pairs_per_step": U_step,
        "keys_last_warmup_step": keys_warm,
        "keys_last_step": status["n_keys"],
        "wall_s_timed": wall,
        "loss_end": loss_end,
        "replay_identical": replay_same,
        "kernels_avg_ms": {k: round(v["avg_ms"], 5) for k, v in sorted(kern.items())},
        "roofline": roofline,
        "kernel_roofline": kernel_roofline,
        "hbm_roofline": hbm,
        "cull": cull,
        "cpu_baseline": cpu,
        "plain": plain,
        "anisotropic": aniso,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
