"""Shared test cases: seeded inputs (from the generator module) and their conditioning.

Conditioning ("boundary-clean" inputs): a pair (voxel, Gaussian) whose Mahalanobis d^2 lies within
``BAND`` of the 3-sigma cutoff 9 can be included by an FP32 evaluation and excluded by the FP64
oracle (or the reverse); both are correct readings of the 3-sigma truncation.  For element-wise
parity the positions of Gaussians owning such a pair are drawn again until no pair is ambiguous.
The check uses the oracle (FP64 d^2), the redraw uses the generator; nothing here comes from the
GPU path.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2603_09621_amd import synth

# |d^2 - 9| band treated as ambiguous between FP32 and FP64 (d^2 units).
BAND = 1e-3


def condition(p: dict, grid: oracle.Grid, seed: int = 12345, band: float = BAND, jitter=None, max_rounds: int = 400):
    """Redraw the positions of Gaussians with ambiguous pairs until none is left."""
    dims = (grid.nx, grid.ny, grid.nz)
    amb = oracle.ambiguous(p, grid, band)
    idx = np.flatnonzero(amb)
    rounds = 0
    while idx.size:
        if rounds >= max_rounds:
            raise RuntimeError(f"conditioning did not converge ({idx.size} Gaussians left)")
        p = synth.redraw_means(p, idx, (seed, rounds), dims, grid.origin, grid.spacing, jitter=jitter)
        amb = oracle.ambiguous(p, grid, band, sel=idx)
        idx = idx[amb > 0]
        rounds += 1
    return p


def condition_obs(p: dict, grid: oracle.Grid, obs, f: int = 4):
    """Observation without sign ties: the fit loss's gradient is sign(zmean(I) - obs), and where
    |zmean(I) - obs| is within the error a correct FP32 render may have in its z-mean
    (``oracle.l1_sign_band``) either sign is correct.  Such observation values are moved to three
    bands from the oracle's z-mean, on the side they were on (below it for an exact tie)."""
    I, _, _ = oracle.render(p, grid)
    return condition_obs_from(I, obs, f)


def condition_obs_from(I, obs, f: int = 4):
    """``condition_obs`` given the oracle's forward I."""
    lr = oracle.zmean(I, f)
    band = oracle.l1_sign_band(I, f)
    obs = np.array(obs, dtype=np.float32, copy=True)
    d = lr - obs.astype(np.float64)
    near = np.abs(d) <= band
    moved = lr[near] - np.where(d[near] >= 0, 3 * band[near], -3 * band[near])
    obs[near] = moved.astype(np.float32)
    assert not oracle.l1_sign_ties(I, obs, f).any()
    return obs


def small_case(seed: int, dims=(20, 18, 12), n: int = 60, ls_mean=None, ls_std=0.3, max_ratio=None,
               cond: bool = True):
    kw = {} if ls_mean is None else {"ls_mean": ls_mean}
    p = synth.gaussians_uniform(seed, n, dims, ls_std=ls_std, max_ratio=max_ratio, **kw)
    grid = oracle.Grid(*dims)
    if cond:
        p = condition(p, grid, seed=seed + 7)
    return p, grid


def plain_case(seed: int = 1, dims=(64, 64, 32), n: int = 20000, cond: bool = True):
    """The plain render + gradient workload (64x64x32, 20k Gaussians, U(0,1) target), conditioned."""
    p, T = synth.workload_plain(seed, dims, n)
    grid = oracle.Grid(*dims)
    if cond:
        p = condition(p, grid, seed=seed + 7)
    return p, T, grid
