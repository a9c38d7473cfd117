"""Parity at the full sizes of the benchmark workloads (sampled or masked comparisons), in the
launch configurations the benchmark times (fit step, batched fit step, batched forward-only render).

Anisotropic backward-heavy workload (320x320x256, 2M Gaussians, log-scale std 0.8, axis ratio <= 8):
inputs cannot be conditioned (the largest Gaussians always have pairs within the FP32/FP64 ambiguity
band of the 3-sigma cutoff), so the forward is compared at every voxel that has no ambiguous pair,
and gradients for 64 sampled Gaussians without ambiguous pairs, stage-wise (both sides take the
oracle's I, W and dL/dI).  Fit workload (256x256x128, 500k Gaussians): forward at 4096 sampled
voxels, and the useful-pair count within the number of ambiguous pairs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_09621_amd import synth
from tests import cases
from tests.gpu_util import assert_fwd_close, assert_grad_close, gpu_grads, gpu_render, np64, say, to_grid

pytestmark = pytest.mark.gpu


def test_anisotropic_workload_full_size():
    p, T = synth.workload_aniso()
    grid = oracle.Grid(320, 320, 256)
    say("aniso full size: GPU render")
    g, ggrid, opts, bins, I, W = gpu_render(p, grid, headroom=1.1)
    Ig, Wg = np64(I), np64(W)
    say("aniso full size: oracle render + ambiguity")
    Io, Wo, _ = oracle.render(p, grid)
    amb = oracle.ambiguous_voxels(p, grid, cases.BAND)
    clean = amb == 0
    say(f"  clean voxels {clean.mean():.3f}")
    assert clean.mean() > 0.5
    assert_fwd_close(Wg[clean], Wo[clean], "aniso W")
    assert_fwd_close(Ig[clean], Io[clean], "aniso I")
    # gradients: 64 sampled Gaussians without ambiguous pairs, stage-wise inputs from the oracle
    per_g = oracle.ambiguous(p, grid, cases.BAND)
    cand = np.flatnonzero(per_g == 0)
    sel = np.sort(np.random.default_rng(7).choice(cand, 64, replace=False))
    _, go = oracle.mse_loss(Io, T)
    I32, W32, g32 = (x.astype(np.float32) for x in (Io, Wo, go))
    del Io, Wo, go
    d = torch.device("cuda")
    say("aniso full size: GPU backward")
    gg = gpu_grads(g, ggrid, opts, bins, torch.from_numpy(I32).to(d), torch.from_numpy(W32).to(d),
                   torch.from_numpy(g32).to(d))
    ref = oracle.grad(p, grid, I32.astype(np.float64), W32.astype(np.float64), g32.astype(np.float64), sel=sel)
    for k in oracle.GROUPS:
        assert_grad_close(gg[k][sel], ref[k][sel], f"aniso d_{k}")


def test_fit_workload_full_size_sampled():
    p, lr_obs, _ = synth.workload_fit()
    grid = oracle.Grid(256, 256, 128)
    say("fit full size: GPU render")
    g, ggrid, opts, bins, I, W = gpu_render(p, grid)
    from paper_2603_09621_amd import gs

    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gs.gs_count_pairs(g, ggrid, opts, bins, cnt)
    vox = np.random.default_rng(8).choice(grid.size, 4096, replace=False)
    amb = oracle.ambiguous_voxels(p, grid, cases.BAND).reshape(-1)
    vox = vox[amb[vox] == 0]
    say(f"fit full size: oracle at {vox.size} voxels")
    Io, Wo, _ = oracle.render_points(p, grid, vox)
    assert_fwd_close(np64(W).reshape(-1)[vox], Wo, "fit W")
    assert_fwd_close(np64(I).reshape(-1)[vox], Io, "fit I")
    n_amb = int(oracle.ambiguous(p, grid, cases.BAND).sum())
    assert abs(int(cnt.item()) - oracle.count_pairs(p, grid)) <= n_amb


def _fit_stagewise_check(gs, p, lr_obs, dims, I_t, W_t, grads, loss, what, nsel=64, seed=9):
    """Stage-wise check of one fit step's loss and gradients at full size: the oracle takes the GPU's
    I and W (FP32) and forms the loss and dL/dI itself; gradients of `nsel` sampled Gaussians without
    ambiguous pairs are compared."""
    grid = oracle.Grid(*dims)
    I = np64(I_t).reshape(grid.shape)
    W = np64(W_t).reshape(grid.shape)
    L, gI = oracle.fit_l1_loss(I, lr_obs, 4)
    assert loss == pytest.approx(L, rel=1e-5), what
    per_g = oracle.ambiguous(p, grid, cases.BAND)
    cand = np.flatnonzero(per_g == 0)
    sel = np.sort(np.random.default_rng(seed).choice(cand, min(nsel, cand.size), replace=False))
    ref = oracle.grad(p, grid, I, W, gI, sel=sel)
    for k in ("mu", "log_scale", "quat", "amp", "relax"):
        got = np64(getattr(grads, k)).reshape(ref[k].shape)
        assert_grad_close(got[sel], ref[k][sel], f"{what} d_{k}",
                          floor=1e-7 * float(np.sqrt(np.mean(ref["mu"][sel] ** 2))))


def test_fit_step_full_size_stagewise():
    """One gs_fit_step of the fit workload (256x256x128, 500k Gaussians) in the benchmark's launch
    configuration: sampled forward voxels, the fused L1 loss and 64 sampled gradients."""
    from paper_2603_09621_amd import gs

    p, lr_obs, _ = synth.workload_fit()
    dims = (256, 256, 128)
    grid = gs.Grid(*dims)
    g = gs.Gaussians.from_numpy(p)
    fo = gs.FitOpts(grid)
    bins = gs.plan_bins(g, grid, fo.opts, headroom=1.5)
    st = gs.FitState(g)
    buf = gs.FitBuffers(g.n, grid, relax=True)
    say("fit step full size")
    gs.gs_fit_step(st, torch.from_numpy(lr_obs).cuda(), fo, bins, buf)
    gs.gs_status(bins)
    og = oracle.Grid(*dims)
    vox = np.sort(np.random.default_rng(10).choice(og.size, 3000, replace=False))
    lo = oracle.render_points(p, og, vox, cutoff=float(np.sqrt(9.0 - cases.BAND)))
    hi = oracle.render_points(p, og, vox, cutoff=float(np.sqrt(9.0 + cases.BAND)))
    clean = (lo[0] == hi[0]) & (lo[1] == hi[1])
    Io, Wo, _ = oracle.render_points(p, og, vox)
    assert_fwd_close(np64(buf.I).reshape(-1)[vox][clean], Io[clean], "fit step I")
    assert_fwd_close(np64(buf.W).reshape(-1)[vox][clean], Wo[clean], "fit step W")
    _fit_stagewise_check(gs, p, lr_obs, dims, buf.I, buf.W, buf.grads, float(buf.loss.item()), "fit step")


def test_batch_full_size_stagewise():
    """One batched fit step of the 16-scan uneven batch (74M voxels, 4.9M Gaussians): every scan's
    forward at sampled voxels and loss, and sampled gradients of the smallest and largest scan."""
    from paper_2603_09621_amd import gs

    scans = synth.workload_batch(seed=4)
    batch = gs.Batch([q["amp"].shape[0] for q, _, _ in scans], [gs.Grid(*d) for _, _, d in scans])
    g = gs.concat([gs.Gaussians.from_numpy(q) for q, _, _ in scans])
    fo = gs.FitOpts(None)
    bins = gs.plan_bins_batch(g, batch, fo.opts, headroom=1.5)
    st = gs.FitState(g, nscans=len(batch))
    buf = gs.FitBuffers(g.n, batch, relax=True, need_dL_dI=False)
    obs = torch.from_numpy(np.concatenate([lr.reshape(-1) for _, lr, _ in scans])).cuda()
    say("batch full size", g.n, batch.v_offsets[-1])
    gs.gs_fit_step_batch(st, obs, batch, fo, bins, buf)
    gs.gs_status(bins)
    Is, Ws = batch.split(buf.I), batch.split(buf.W)
    losses = buf.loss.cpu().numpy()
    rng = np.random.default_rng(11)
    for k, (q, lr, d) in enumerate(scans):
        og = oracle.Grid(*d)
        vox = np.sort(rng.choice(og.size, 400, replace=False))
        lo = oracle.render_points(q, og, vox, cutoff=float(np.sqrt(9.0 - cases.BAND)))
        hi = oracle.render_points(q, og, vox, cutoff=float(np.sqrt(9.0 + cases.BAND)))
        clean = (lo[0] == hi[0]) & (lo[1] == hi[1])
        Io, _, _ = oracle.render_points(q, og, vox)
        assert_fwd_close(np64(Is[k]).reshape(-1)[vox][clean], Io[clean], f"batch scan {k} I")
        L, _ = oracle.fit_l1_loss(np64(Is[k]), lr, 4)
        assert float(losses[k]) == pytest.approx(L, rel=1e-5), f"batch scan {k} loss"
    sizes = [d[0] * d[1] * d[2] for _, _, d in scans]
    o = batch.g_offsets
    for k in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        q, lr, d = scans[k]
        sub = gs.Grads(*(None if getattr(buf.grads, n) is None else getattr(buf.grads, n)[o[k]:o[k + 1]]
                         for n in gs.GROUPS))
        say(f"  batch scan {k} {d}: sampled gradients")
        _fit_stagewise_check(gs, q, lr, d, Is[k], Ws[k], sub, float(losses[k]), f"batch scan {k}", nsel=32)


def test_serving_set_full_size_render():
    """The largest resident set of the request-loop workload rendered at scale 4 of its LR box through
    the request loop's batched forward-only path (with a second set in the same batch), sampled
    voxels vs the oracle."""
    from paper_2603_09621_amd import gs

    sets = synth.serving_sets(5, 32)
    order = np.argsort([q["amp"].shape[0] for q, _ in sets])
    picks = [sets[order[-1]], sets[order[0]]]
    grids = [gs.Grid.at_scale(picks[0][1], 4.0), gs.Grid.at_scale(picks[1][1], 2.5)]
    gsets = [gs.Gaussians.from_numpy(q) for q, _ in picks]
    batch = gs.Batch.of_sets(gsets, grids)
    opts = gs.Opts(forward_only=True)
    say("serving set full size", [x.n for x in gsets], [gr.shape for gr in grids])
    I, _, bins = gs.render_batch(None, batch, opts, want_w=False)
    gs.gs_status(bins)
    rng = np.random.default_rng(12)
    for k, ((q, _), gr) in enumerate(zip(picks, grids)):
        og = oracle.Grid(gr.nx, gr.ny, gr.nz, gr.origin, gr.spacing)
        vox = np.sort(rng.choice(og.size, 1500, replace=False))
        lo = oracle.render_points(q, og, vox, cutoff=float(np.sqrt(9.0 - cases.BAND)))
        hi = oracle.render_points(q, og, vox, cutoff=float(np.sqrt(9.0 + cases.BAND)))
        clean = (lo[0] == hi[0]) & (lo[1] == hi[1])
        Io, _, _ = oracle.render_points(q, og, vox)
        assert clean.mean() > 0.9
        assert_fwd_close(np64(batch.split(I)[k]).reshape(-1)[vox][clean], Io[clean], f"serving set {k} I")
