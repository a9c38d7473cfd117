"""PSNR / SSIM used for the fit sanity checks, pinned against their definitions (CPU)."""
import math

import numpy as np

from paper_2603_09621_amd import metrics


def test_psnr_definition():
    ref = np.zeros((4, 5, 6))
    ref[0, 0, 0] = 1.0  # data range 1
    x = ref + 0.1  # MSE 0.01 -> 20 dB
    assert math.isclose(metrics.psnr(x, ref), 20.0, rel_tol=1e-12)
    assert metrics.psnr(ref, ref) == float("inf")
    assert math.isclose(metrics.psnr(x, ref, data_range=10.0), 40.0, rel_tol=1e-12)


def test_ssim_identity_and_symmetry():
    rng = np.random.default_rng(0)
    a = rng.random((12, 13, 14))
    b = a + 0.1 * rng.standard_normal(a.shape)
    assert metrics.ssim(a, a) == 1.0 or math.isclose(metrics.ssim(a, a), 1.0, rel_tol=1e-12)
    assert math.isclose(metrics.ssim(a, b, data_range=1.0), metrics.ssim(b, a, data_range=1.0), rel_tol=1e-12)
    assert metrics.ssim(a, b, data_range=1.0) < 1.0


def test_ssim_matches_explicit_window_sum():
    """One interior voxel of the SSIM map against the weighted sums written out with an explicit
    normalised Gaussian window."""
    rng = np.random.default_rng(1)
    x = rng.random((15, 15, 15))
    y = 0.7 * x + 0.3 * rng.random(x.shape)
    sig, trunc = 1.5, 3.5
    rad = int(trunc * sig + 0.5)
    o = np.arange(-rad, rad + 1)
    g1 = np.exp(-0.5 * (o / sig) ** 2)
    g1 /= g1.sum()
    w = g1[:, None, None] * g1[None, :, None] * g1[None, None, :]
    c = 7
    sl = tuple(slice(c - rad, c + rad + 1) for _ in range(3))
    px, py = x[sl], y[sl]
    mx, my = (w * px).sum(), (w * py).sum()
    vx = (w * px * px).sum() - mx * mx
    vy = (w * py * py).sum() - my * my
    cxy = (w * px * py).sum() - mx * my
    r = 1.0
    c1, c2 = (0.01 * r) ** 2, (0.03 * r) ** 2
    want = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    got = metrics.ssim_map(x, y, data_range=1.0)[c, c, c]
    assert math.isclose(got, want, rel_tol=1e-10)


def test_ssim_of_scaled_constant_volumes():
    """Constant volumes a and b: SSIM = (2ab + C1) / (a^2 + b^2 + C1) (all variances vanish)."""
    a, b = 0.4, 0.6
    x = np.full((9, 9, 9), a)
    y = np.full((9, 9, 9), b)
    c1 = 0.01 ** 2
    assert math.isclose(metrics.ssim(x, y, data_range=1.0), (2 * a * b + c1) / (a * a + b * b + c1), rel_tol=1e-9)
