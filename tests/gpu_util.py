"""Helpers for the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle

FWD_RTOL, FWD_ATOL = 1e-5, 1e-7
GRAD_RTOL, GRAD_RMS = 1e-4, 1e-4


def gs_mod():
    from paper_2603_09621_amd import gs  # noqa: WPS433 (imported lazily: needs the built library)
    return gs


def say(*a):
    print("[gpu]", *a, flush=True)


def to_grid(grid: oracle.Grid):
    gs = gs_mod()
    return gs.Grid(grid.nx, grid.ny, grid.nz, tuple(grid.origin), tuple(grid.spacing))


def gpu_render(p: dict, grid: oracle.Grid, cutoff=3.0, eps=1e-8, headroom=1.25):
    gs = gs_mod()
    g = gs.Gaussians.from_numpy(p)
    ggrid = to_grid(grid)
    opts = gs.Opts(cutoff=cutoff, eps=eps)
    I, W, bins = gs.render(g, ggrid, opts)
    gs.gs_status(bins)
    return g, ggrid, opts, bins, I, W


def gpu_grads(g, ggrid, opts, bins, I, W, gI):
    gs = gs_mod()
    grads = gs.backward(g, ggrid, opts, bins, I, W, gI)
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy().astype(np.float64)) for k, v in grads.as_dict().items()}


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def assert_fwd_close(x, y, what=""):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    err = np.abs(x - y)
    lim = FWD_RTOL * np.abs(y) + FWD_ATOL
    bad = err > lim
    if bad.any():
        i = np.flatnonzero(bad.reshape(-1))[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} elements off; worst rel "
                             f"{float(np.max(err / (np.abs(y) + 1e-30))):.3e}; first idx {i} got "
                             f"{x.reshape(-1)[i]} want {y.reshape(-1)[i]}")


def assert_grad_close(x, y, what="", floor=0.0):
    """|x - y| <= 1e-4 |y| + 1e-4 rms(y) + floor (floor: for arrays whose exact value is 0 by
    symmetry, where y holds only rounding noise)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    rms = float(np.sqrt(np.mean(y * y))) if y.size else 0.0
    err = np.abs(x - y)
    lim = GRAD_RTOL * np.abs(y) + GRAD_RMS * rms + floor
    bad = err > lim
    if bad.any():
        i = np.flatnonzero(bad.reshape(-1))[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} entries off (rms {rms:.3e}); got "
                             f"{x.reshape(-1)[i]} want {y.reshape(-1)[i]}")


def rel_l2(x, y) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))
