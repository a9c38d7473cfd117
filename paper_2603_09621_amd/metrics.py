"""Image-quality metrics for sanity checks of fitted volumes (§4 reports PSNR and SSIM).

Host-side numpy/scipy on volumes copied from the device; not part of the rendering path.

* PSNR = 10 log10(R^2 / MSE) with R the data range (default: max - min of the reference).
* SSIM (Wang et al. 2004), 3-D: local means, variances and covariance from a Gaussian window
  (sigma 1.5 voxels, truncated at 3.5 sigma, reflect padding), C1 = (0.01 R)^2, C2 = (0.03 R)^2,
  SSIM = mean over voxels of (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)).
"""
from __future__ import annotations

from typing import Optional

import numpy as np
from scipy import ndimage


def psnr(x, ref, data_range: Optional[float] = None) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    r = float(ref.max() - ref.min()) if data_range is None else float(data_range)
    mse = float(np.mean((x - ref) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(r * r / mse)


def ssim_map(x, ref, data_range: Optional[float] = None, sigma: float = 1.5, truncate: float = 3.5):
    x = np.asarray(x, np.float64)
    y = np.asarray(ref, np.float64)
    r = float(y.max() - y.min()) if data_range is None else float(data_range)
    c1, c2 = (0.01 * r) ** 2, (0.03 * r) ** 2

    def f(a):
        return ndimage.gaussian_filter(a, sigma, mode="reflect", truncate=truncate)

    mx, my = f(x), f(y)
    sxx = f(x * x) - mx * mx
    syy = f(y * y) - my * my
    sxy = f(x * y) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(x, ref, data_range: Optional[float] = None, sigma: float = 1.5) -> float:
    return float(np.mean(ssim_map(x, ref, data_range, sigma)))
