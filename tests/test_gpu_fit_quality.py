"""Sanity of the per-scan fit on a synthetic phantom (§4 reports PSNR / SSIM of the fitted HR
volume): the L1 data term falls, and the HR render approaches the clean phantom, beating the
starting render and a nearest-neighbour z-upsampling of the LR observation."""
import numpy as np
import pytest
import torch

from paper_2603_09621_amd import metrics, synth
from tests.gpu_util import gs_mod, say

pytestmark = pytest.mark.gpu


def test_fit_improves_psnr_and_ssim():
    gs = gs_mod()
    dims, f, seed = (64, 64, 32), 4, 51
    clean = synth.phantom(seed, dims, noise=0.0)
    noisy = synth.phantom(seed, dims)
    lr = synth.zmean_observation(noisy, f)
    p = synth.lattice_init(seed + 1, lr, (dims[0] // 2) * (dims[1] // 2) * (dims[2] // f), f)
    g = gs.Gaussians.from_numpy(p)
    grid = gs.Grid(*dims)
    fo = gs.FitOpts(grid, zdown=f)
    bins = gs.plan_bins(g, grid, fo.opts, headroom=2.0)
    st = gs.FitState(g)
    buf = gs.FitBuffers(g.n, grid, relax=True)
    obs = torch.from_numpy(lr).cuda()
    losses, curve = [], []
    for it in range(400):
        gs.gs_fit_step(st, obs, fo, bins, buf)
        if it % 50 == 0 or it == 399:
            gs.gs_status(bins)
            losses.append(float(buf.loss.item()))
            curve.append(metrics.psnr(buf.I.cpu().numpy(), clean, data_range=1.0))
        if it == 0:
            first = buf.I.cpu().numpy()
    I, _, b2 = gs.render(g, grid, fo.opts)
    gs.gs_status(b2)
    fit = I.cpu().numpy()
    nearest = np.repeat(lr, f, axis=0)
    q = {name: (metrics.psnr(v, clean, data_range=1.0), metrics.ssim(v, clean, data_range=1.0))
         for name, v in (("start", first), ("fit", fit), ("nearest_z", nearest))}
    say("losses", [round(x, 5) for x in losses])
    say("psnr curve", [round(x, 2) for x in curve])
    say("psnr/ssim", {k: (round(a, 2), round(b, 4)) for k, (a, b) in q.items()})
    assert losses[-1] < 0.5 * losses[0]
    assert q["fit"][0] > q["start"][0] + 3.0
    assert q["fit"][1] > q["start"][1]
    assert q["fit"][0] > q["nearest_z"][0]
