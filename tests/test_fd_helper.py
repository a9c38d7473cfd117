"""The box-local finite difference used at full size equals the whole-grid frozen-support difference
and approaches the oracle's analytic gradient (CPU)."""
import numpy as np

import oracle
from paper_2603_09621_amd import synth
from tests import cases, fd


def test_box_fd_equals_whole_grid_fd_and_gradient():
    p, grid = cases.small_case(51, dims=(22, 20, 16), n=90, ls_std=0.6, max_ratio=6.0)
    p["relax"] = np.random.default_rng(51).uniform(0.5, 1.0, 90).astype(np.float32)
    T = synth.uniform_volume(52, (grid.nx, grid.ny, grid.nz))
    I, W, S = oracle.render(p, grid)
    _, gI = oracle.mse_loss(I, T)
    an = oracle.grad(p, grid, I, W, gI)
    rng = np.random.default_rng(53)
    checked = 0
    for j in rng.choice(90, 24, replace=False):
        key, comp = fd.ENTRIES[rng.integers(len(fd.ENTRIES))]
        r = fd.box_fd_checked(p, grid, S, W, T, int(j), key, comp)
        if r is None:
            continue
        d, trunc = r
        # the same difference over the whole grid with the frozen-support forward
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        x0 = float(p[key].reshape(90, -1)[j, comp])
        pp[key].reshape(90, -1)[j, comp] = np.float32(x0 + fd.H)
        pm[key].reshape(90, -1)[j, comp] = np.float32(x0 - fd.H)
        Ip, _ = oracle.render_frozen(pp, p, grid)
        Im, _ = oracle.render_frozen(pm, p, grid)
        Lp, Lm = float(np.mean((Ip - T) ** 2)), float(np.mean((Im - T) ** 2))
        whole = (Lp - Lm) / (2 * fd.H)
        scale = float(np.sqrt(np.mean(an[key] ** 2)))
        # the whole-grid difference cancels two losses of size L: its own rounding is ~u L / h
        assert abs(d - whole) <= 1e-9 * abs(whole) + 64 * 2.0 ** -53 * Lp / fd.H, (key, comp, d, whole)
        a = float(an[key].reshape(90, -1)[j, comp])
        assert abs(d - a) <= 1e-6 * abs(a) + trunc + 1e-9 * scale, (key, comp, d, a, trunc)
        checked += 1
    assert checked >= 20
