"""The autograd.Function over the forward/backward kernels: gradients of a scalar loss against the
oracle's analytic gradient and against central finite differences of the oracle's frozen-support
forward (FP64), on the anisotropic workload's distribution (log-scale std 0.8, axis ratio <= 8)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2603_09621_amd import synth
from tests import cases
from tests.gpu_util import assert_grad_close, say, to_grid

pytestmark = pytest.mark.gpu


def _tensors(p, requires_grad=True):
    return [torch.tensor(p[k], device="cuda", requires_grad=requires_grad) for k in oracle.GROUPS]


def test_autograd_matches_oracle_gradient():
    from paper_2603_09621_amd import autograd

    p, grid = cases.small_case(41, dims=(40, 36, 24), n=600, ls_std=0.8, max_ratio=8.0)
    p["relax"] = np.random.default_rng(41).uniform(0.4, 1.0, 600).astype(np.float32)
    T = synth.uniform_volume(42, (grid.nx, grid.ny, grid.nz))
    say("autograd vs oracle", grid.shape)
    ts = _tensors(p)
    I = autograd.render(*ts, to_grid(grid))
    loss = ((I - torch.from_numpy(T).cuda()) ** 2).mean()
    loss.backward()
    Io, Wo, _ = oracle.render(p, grid)
    _, go = oracle.mse_loss(Io, T)
    ref = oracle.grad(p, grid, Io, Wo, go)
    for k, t in zip(oracle.GROUPS, ts):
        assert_grad_close(t.grad.cpu().numpy(), ref[k], f"autograd d_{k}")


def test_autograd_matches_frozen_support_finite_differences():
    """64 random parameter entries (every group, the relaxation factor included), h = 1e-3: the GPU
    gradient of L = <g, I> equals the central difference of the oracle's FP64 forward with the
    support held fixed."""
    from paper_2603_09621_amd import autograd

    p, grid = cases.small_case(43, dims=(32, 28, 20), n=300, ls_std=0.8, max_ratio=8.0)
    p["relax"] = np.random.default_rng(43).uniform(0.4, 1.0, 300).astype(np.float32)
    g = np.random.default_rng(44).standard_normal(grid.shape)
    say("autograd vs finite differences", grid.shape)
    ts = _tensors(p)
    I = autograd.render(*ts, to_grid(grid))
    (I * torch.from_numpy(g.astype(np.float32)).cuda()).sum().backward()
    an = {k: t.grad.cpu().numpy().astype(np.float64) for k, t in zip(oracle.GROUPS, ts)}
    rng = np.random.default_rng(45)
    h = 1e-3
    for _ in range(64):
        k = oracle.GROUPS[rng.integers(len(oracle.GROUPS))]
        j = int(rng.integers(p[k].size))
        pp = {kk: vv.copy() for kk, vv in p.items()}
        pm = {kk: vv.copy() for kk, vv in p.items()}
        pp[k].reshape(-1)[j] = np.float32(p[k].reshape(-1)[j] + h)
        pm[k].reshape(-1)[j] = np.float32(p[k].reshape(-1)[j] - h)
        step = float(pp[k].reshape(-1)[j]) - float(pm[k].reshape(-1)[j])
        fd = float(((oracle.render_frozen(pp, p, grid)[0] - oracle.render_frozen(pm, p, grid)[0]) * g).sum()) / step
        a = float(an[k].reshape(-1)[j])
        scale = float(np.abs(an[k]).max())
        assert abs(fd - a) <= 1e-3 * abs(a) + 1e-4 * scale, (k, j, fd, a)
