"""Rendering a fitted-set-like Gaussian set at arbitrary target shapes (§4.2: the representation is
rendered at any requested grid), at the full sizes of the paper's two datasets' volumes: a brain
MRI-like 240 x 240 x 155 grid and a fetal MRI-like 256 x 256 x 256 grid, both from an anisotropic LR
box (non-uniform scale factors).  Sampled voxels are compared with the oracle evaluated at those
voxels; a sampled voxel is used only if the oracle gives bitwise the same result at cutoffs
sqrt(9 - band) and sqrt(9 + band) (no pair within the FP32/FP64 ambiguity band there)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2603_09621_amd import synth
from tests import cases
from tests.gpu_util import assert_fwd_close, gs_mod, say

pytestmark = pytest.mark.gpu

SHAPES = {
    # name: (LR box (x, y, z) in LR voxels, target shape (nx, ny, nz), Gaussians)
    "brain_240x240x155": ((120, 120, 39), (240, 240, 155), 150000),
    "fetal_256x256x256": ((128, 128, 64), (256, 256, 256), 200000),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_render_at_dataset_shapes(name):
    gs = gs_mod()
    box, shape, n = SHAPES[name]
    ell = (np.prod(box) / n) ** (1 / 3)
    p = synth.gaussians_uniform(61, n, box, ls_mean=float(math.log(0.8 * ell)), ls_std=0.3, max_ratio=4.0)
    p["relax"] = np.random.default_rng(62).uniform(0.5, 1.0, n).astype(np.float32)
    sp = tuple(b / s for b, s in zip(box, shape))
    grid = gs.Grid(*shape, origin=tuple(0.5 * s for s in sp), spacing=sp)
    og = oracle.Grid(*shape, grid.origin, grid.spacing)
    say("shape", name, shape, n)
    g = gs.Gaussians.from_numpy(p)
    I, W, bins = gs.render(g, grid, gs.Opts())
    gs.gs_status(bins)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gs.gs_count_pairs(g, grid, gs.Opts(), bins, cnt)
    rng = np.random.default_rng(63)
    vox = np.sort(rng.choice(grid.size, size=6000, replace=False))
    lo = oracle.render_points(p, og, vox, cutoff=math.sqrt(9.0 - cases.BAND))
    hi = oracle.render_points(p, og, vox, cutoff=math.sqrt(9.0 + cases.BAND))
    Io, Wo, _ = oracle.render_points(p, og, vox)
    clean = (lo[0] == hi[0]) & (lo[1] == hi[1])
    say("  clean sampled voxels", int(clean.sum()), "of", vox.size, "pairs", int(cnt.item()))
    assert clean.sum() > 0.9 * vox.size
    Ig = I.reshape(-1)[torch.from_numpy(vox).cuda()].cpu().numpy()
    Wg = W.reshape(-1)[torch.from_numpy(vox).cuda()].cpu().numpy()
    assert_fwd_close(Wg[clean], Wo[clean], f"{name} W")
    assert_fwd_close(Ig[clean], Io[clean], f"{name} I")
