"""Box-local central differences of the MSE loss in one parameter of one Gaussian, with the support
held fixed (test helper, CPU).

L = mean_p (I(p) - T(p))^2.  Changing one parameter of Gaussian j changes I only inside j's padded
index box, where I(p) = (S_o(p) + A_j w_j(p)) / (W_o(p) + w_j(p) + eps), S_o and W_o being the sums
of the other Gaussians (the oracle's full forward minus j's own terms).  So the difference
L(theta + h) - L(theta - h) is a sum over the box alone, written as
sum (I+ - I-)(I+ + I- - 2 T) / V so that nothing large cancels.  The perturbed values are FP32
parameters; h is a power of two so that theta +- h are exact and the difference is central.
"""
from __future__ import annotations

import numpy as np

import oracle

H = 2.0 ** -10  # ~1e-3, exactly representable


def box_fd_mse(p: dict, grid: oracle.Grid, S, W, T, j: int, key: str, comp: int, h: float = H, eps: float = 1e-8):
    """Central difference of the MSE loss in entry ``comp`` of ``p[key]`` of Gaussian j.  S, W: the
    oracle's forward of p (float64, [nz, ny, nx]); T: the target.  Returns None if theta +- h is not
    exact in FP32 (then pick another entry)."""
    one = {k: np.asarray(v)[j:j + 1].copy() for k, v in p.items() if v is not None}
    vox, w0 = oracle.weights_box(one, 0, grid)
    A0 = float(one["amp"][0])
    So = S.reshape(-1)[vox] - A0 * w0
    Wo = W.reshape(-1)[vox] - w0
    Tv = np.asarray(T, dtype=np.float64).reshape(-1)[vox]
    x0 = float(one[key].reshape(-1)[comp])
    Ipm = []
    for sgn in (1.0, -1.0):
        q = {k: v.copy() for k, v in one.items()}
        flat = q[key].reshape(-1)
        flat[comp] = np.float32(x0 + sgn * h)
        if float(flat[comp]) - x0 != sgn * h:
            return None
        _, w = oracle.weights_box(q, 0, grid, support=one)
        Ipm.append((So + float(q["amp"][0]) * w) / (Wo + w + eps))
    Ip, Im = Ipm
    return float(np.sum((Ip - Im) * (Ip + Im - 2.0 * Tv))) / (grid.size * 2.0 * h)


def box_fd_checked(p, grid, S, W, T, j, key, comp, h: float = H):
    """(difference at h, its truncation allowance 4/3 |D(h) - D(h/2)|), or None."""
    a = box_fd_mse(p, grid, S, W, T, j, key, comp, h)
    b = box_fd_mse(p, grid, S, W, T, j, key, comp, h / 2)
    if a is None or b is None:
        return None
    return a, 4.0 / 3.0 * abs(a - b)


ENTRIES = [(k, c) for k, n in (("mu", 3), ("log_scale", 3), ("quat", 4), ("amp", 1), ("relax", 1)) for c in range(n)]
