"""Seeded synthetic inputs: Gaussian sets, targets, MRI-like phantoms, LR observations, lattice
initialisation.

This module draws random numbers and lays them out; it holds none of the renderer's arithmetic
(no weights, no Mahalanobis distances, no normalised aggregation).  Both the GPU path and the
oracle consume the arrays it returns, so it imports neither of them.  Every array is FP32, volumes
are [nz][ny][nx] (x fastest) and positions are in world units with voxel (ix, iy, iz) centred at
origin + spacing * (ix, iy, iz); the default grid has origin 0.5 and spacing 1, so a volume of
dims (nx, ny, nz) spans [0, nx) x [0, ny) x [0, nz).

Workload recipes (the paper's MRI volumes are not available; these stand in for them):
  * ``gaussians_uniform``: mu ~ U(volume), natural-log scales ~ N(ln 1.5, std) per axis (optionally
    redrawn until the axis ratio max/min sigma <= max_ratio), uniform random unit quaternions (four
    i.i.d. N(0,1) normalised), amplitude ~ U(0,1), relaxation r = 1.
  * ``phantom``: 60 random soft ellipsoids composited over 0 with smooth-edged masks and intensities
    in [0.1, 1], plus i.i.d. N(0, noise^2) noise.
  * ``zmean_observation``: the LR scan as the mean of groups of 4 consecutive z slices.
  * ``lattice_init``: Gaussians initialised from the coordinates of the LR volume (Fig. 1 caption).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Tuple

import numpy as np

LN15 = math.log(1.5)


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (w, x, y, z): four i.i.d. N(0,1) draws, normalised."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def log_scales(rng: np.random.Generator, n: int, mean: float = LN15, std: float = 0.3,
               max_ratio: Optional[float] = None) -> np.ndarray:
    """Natural-log scales ~ N(mean, std) per axis; with ``max_ratio``, each Gaussian's triple is
    redrawn until max sigma / min sigma <= max_ratio."""
    s = rng.normal(mean, std, (n, 3))
    if max_ratio is not None:
        lim = math.log(max_ratio)
        bad = np.flatnonzero(s.max(axis=1) - s.min(axis=1) > lim)
        while bad.size:
            s[bad] = rng.normal(mean, std, (bad.size, 3))
            bad = bad[s[bad].max(axis=1) - s[bad].min(axis=1) > lim]
    return s.astype(np.float32)


def gaussians_uniform(seed, n: int, dims: Sequence[int], ls_mean: float = LN15, ls_std: float = 0.3,
                      max_ratio: Optional[float] = None, origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0)) -> dict:
    """n Gaussians with mu uniform over the grid's extent [origin - spacing/2, ... + dims*spacing)."""
    rng = _rng(seed)
    dims = np.asarray(dims, dtype=np.float64)
    lo = np.asarray(origin) - 0.5 * np.asarray(spacing)
    ext = dims * np.asarray(spacing)
    mu = (lo + rng.random((n, 3)) * ext).astype(np.float32)
    ls = log_scales(rng, n, ls_mean, ls_std, max_ratio)
    q = random_quaternions(rng, n)
    amp = rng.random(n).astype(np.float32)
    relax = np.ones(n, dtype=np.float32)
    return {"mu": mu, "log_scale": ls, "quat": q, "amp": amp, "relax": relax}


def redraw_means(p: dict, idx, seed, dims: Sequence[int], origin=(0.5, 0.5, 0.5), spacing=(1.0, 1.0, 1.0),
                 jitter: Optional[Sequence[float]] = None) -> dict:
    """Copy of ``p`` with the positions of Gaussians ``idx`` drawn again (uniform over the grid, or,
    with ``jitter``, the old position plus U(-1/2, 1/2) * jitter per axis)."""
    rng = _rng(seed)
    idx = np.asarray(idx, dtype=np.int64)
    out = {k: np.array(v, copy=True) for k, v in p.items()}
    if idx.size == 0:
        return out
    if jitter is None:
        lo = np.asarray(origin) - 0.5 * np.asarray(spacing)
        ext = np.asarray(dims, dtype=np.float64) * np.asarray(spacing)
        out["mu"][idx] = (lo + rng.random((idx.size, 3)) * ext).astype(np.float32)
    else:
        out["mu"][idx] = (out["mu"][idx] + (rng.random((idx.size, 3)) - 0.5) * np.asarray(jitter)).astype(
            np.float32)
    return out


def uniform_volume(seed, dims: Sequence[int]) -> np.ndarray:
    """i.i.d. U(0,1) volume of dims (nx, ny, nz), stored [nz][ny][nx]."""
    nx, ny, nz = dims
    return _rng(seed).random((nz, ny, nx), dtype=np.float32)


def phantom(seed, dims: Sequence[int], n_ellipsoids: int = 60, noise: float = 0.01, edge: float = 0.05) -> np.ndarray:
    """MRI-like synthetic volume of dims (nx, ny, nz), [nz][ny][nx] FP32.

    Ellipsoid j: centre U(0.15, 0.85) * dims, semi-axes U(0.04, 0.25) * dims (per axis), uniform
    random rotation, intensity U(0.1, 1).  Its mask is m_j = sigmoid((1 - rho_j) / edge) with rho_j
    the ellipsoidal radius, set to exactly 0 where rho_j > 2 (there m_j < 3e-9).  Masks are
    composited in index order over 0 (V <- V (1 - m_j) + c_j m_j), so the clean volume lies in
    [0, 1]; then i.i.d. N(0, noise^2) noise is added (not clipped)."""
    rng = _rng(seed)
    nx, ny, nz = (int(d) for d in dims)
    dimv = np.array([nx, ny, nz], dtype=np.float64)
    V = np.zeros((nz, ny, nx), dtype=np.float32)
    for _ in range(n_ellipsoids):
        c = rng.uniform(0.15, 0.85, 3) * dimv
        ax = rng.uniform(0.04, 0.25, 3) * dimv
        qq = rng.standard_normal(4)
        qq /= np.linalg.norm(qq)
        w, x, y, z = qq
        rot = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        val = rng.uniform(0.1, 1.0)
        # bounding box of the rho <= 2 region
        half = 2.0 * np.sqrt(((rot * ax[None, :]) ** 2).sum(axis=1))
        lo = np.maximum(np.floor(c - half - 0.5).astype(int), 0)
        hi = np.minimum(np.ceil(c + half - 0.5).astype(int) + 1, [nx, ny, nz])
        if np.any(hi <= lo):
            continue
        zs = np.arange(lo[2], hi[2], dtype=np.float32) + 0.5 - c[2]
        ys = np.arange(lo[1], hi[1], dtype=np.float32) + 0.5 - c[1]
        xs = np.arange(lo[0], hi[0], dtype=np.float32) + 0.5 - c[0]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        # coordinates in the ellipsoid's own frame: u = rot^T (p - c)
        rho2 = np.zeros_like(X)
        for k in range(3):
            u = X * np.float32(rot[0, k]) + Y * np.float32(rot[1, k]) + Z * np.float32(rot[2, k])
            rho2 += (u / np.float32(ax[k])) ** 2
        rho = np.sqrt(rho2)
        with np.errstate(over="ignore"):  # exp overflows to inf far outside: m = 0 there
            m = (1.0 / (1.0 + np.exp(-(1.0 - rho) / edge))).astype(np.float32)
        m[rho > 2.0] = 0.0
        sub = V[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub *= (1.0 - m)
        sub += np.float32(val) * m
    V += (noise * rng.standard_normal(V.shape)).astype(np.float32)
    return V


def zmean_observation(hr: np.ndarray, f: int = 4) -> np.ndarray:
    """LR observation of a HR volume: mean of each group of f consecutive z slices (FP32)."""
    nz, ny, nx = hr.shape
    assert nz % f == 0, "nz must be a multiple of the z factor"
    return hr.astype(np.float64).reshape(nz // f, f, ny, nx).mean(axis=1).astype(np.float32)


def lattice_init(seed, lr_obs: np.ndarray, n: int, f: int = 4, stride_xy: int = 2, jitter: bool = True) -> dict:
    """Gaussians initialised from the coordinates of the LR volume (zero-shot, Fig. 1 caption).

    Sites are LR voxel centres on an in-plane lattice of stride ``stride_xy`` (HR frame: x = s*a + s/2,
    y = s*b + s/2, z = f*k + f/2, i.e. the centre of the s x s x f block of HR voxels); ``n`` of them
    are chosen without replacement, each jittered by U(-1/2, 1/2) times the lattice spacing
    (s, s, f).  sigma = half the lattice spacing (log-scales ln(s/2), ln(s/2), ln(f/2)); identity
    rotation; amplitude = the LR value at the site's first voxel; r = 1."""
    rng = _rng(seed)
    nzl, ny, nx = lr_obs.shape
    s = stride_xy
    ax, by, kz = nx // s, ny // s, nzl
    sites = ax * by * kz
    if n > sites:
        raise ValueError(f"lattice has {sites} sites, fewer than n={n}")
    pick = np.sort(rng.choice(sites, size=n, replace=False))
    k = pick // (ax * by)
    b = (pick // ax) % by
    a = pick % ax
    mu = np.stack([s * a + s / 2.0, s * b + s / 2.0, f * k + f / 2.0], axis=1)
    if jitter:
        mu = mu + (rng.random((n, 3)) - 0.5) * np.array([s, s, f], dtype=np.float64)
    ls = np.tile(np.log(np.array([s / 2.0, s / 2.0, f / 2.0])), (n, 1))
    q = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    amp = lr_obs[k, s * b, s * a]
    return {"mu": mu.astype(np.float32), "log_scale": ls.astype(np.float32), "quat": q.astype(np.float32),
            "amp": np.asarray(amp, dtype=np.float32), "relax": np.ones(n, dtype=np.float32)}


# ------------------------------------------------------------------------------------------------
# Named workloads.

def workload_plain(seed: int = 1, dims=(64, 64, 32), n: int = 20000) -> Tuple[dict, np.ndarray]:
    """Plain render + gradient: dims 64x64x32, 20k Gaussians, target ~ U(0,1) i.i.d., MSE loss."""
    p = gaussians_uniform(seed, n, dims)
    T = uniform_volume(seed + 1000, dims)
    return p, T


def workload_fit(seed: int = 2, dims=(256, 256, 128), n: int = 500000, f: int = 4):
    """Single-scan zero-shot fit: phantom HR (with noise) -> LR observation (z-mean of f) ->
    lattice init with n Gaussians.  Returns (params, lr_obs, hr_noisy)."""
    hr = phantom(seed, dims)
    lr = zmean_observation(hr, f)
    p = lattice_init(seed + 1, lr, n, f)
    return p, lr, hr


def workload_aniso(seed: int = 3, dims=(320, 320, 256), n: int = 2000000):
    """Backward-heavy anisotropic case: log-scale std 0.8, axis ratio <= 8, target ~ U(0,1)."""
    p = gaussians_uniform(seed, n, dims, ls_std=0.8, max_ratio=8.0)
    T = uniform_volume(seed + 1000, dims)
    return p, T


def _round_to(x: float, m: int) -> int:
    return max(m, int(round(x / m)) * m)


def batch_dims(j: int, nscans: int = 16):
    """Grid of scan j of the uneven batch: nx = ny = round_8(96 + 160 j / (S - 1)),
    nz = round_4(96 + 64 j / (S - 1))."""
    t = j / max(nscans - 1, 1)
    nxy = _round_to(96 + 160 * t, 8)
    return (nxy, nxy, _round_to(96 + 64 * t, 4))


def lattice_stride(lr_shape, n: int) -> int:
    """Largest in-plane lattice stride whose site count is still >= n (at least 1)."""
    nzl, ny, nx = lr_shape
    s = 1
    while (nx // (s + 1)) * (ny // (s + 1)) * nzl >= n:
        s += 1
    return s


def workload_batch(seed: int = 4, nscans: int = 16, f: int = 4, n_range=(5e4, 8e5), workers: int = 8):
    """Batch of uneven single-scan fits.  Scan j (before shuffling) has the grid of batch_dims(j);
    its Gaussian count is exp(U(ln lo, ln hi)) (drawn with ``seed``), capped at the number of LR
    voxels (a stride-1 lattice); its HR phantom uses seed 100 + j, its LR observation is the z-mean of
    f, and its Gaussians sit on the coarsest in-plane lattice with enough sites (lattice_init, seed
    200 + j).  The scan order is shuffled with ``seed``.  Returns a list of (params, lr_obs, dims)."""
    rng = _rng(seed)
    ns = np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), nscans))
    order = rng.permutation(nscans)

    def one(j):
        dims = batch_dims(int(j), nscans)
        hr = phantom(100 + int(j), dims)
        lr = zmean_observation(hr, f)
        n = int(min(round(ns[j]), lr.size))
        p = lattice_init(200 + int(j), lr, n, f, stride_xy=lattice_stride(lr.shape, n))
        return p, lr, dims

    # each scan has its own generators, so running them on threads changes nothing
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(one, order))


def serving_sets(seed: int = 5, count: int = 32, n_range=(1e5, 2e6), box_xy=(48, 80), box_z=(32, 48)):
    """Resident Gaussian sets of the request loop.  Per set: N = exp(U(ln lo, ln hi)); LR box
    nx = ny ~ U{box_xy}, nz ~ U{box_z} (LR voxels of unit spacing, centres at 0.5, 1.5, ...);
    mu ~ U(box); log-scales ~ N(ln(0.75 l), 0.3) per axis with l = (V_LR / N)^(1/3) (the mean
    spacing of the Gaussians); uniform random rotations; A ~ U(0, 1); r = 1.  Set k uses seed
    (seed, k).  Returns a list of (params, (nx, ny, nz))."""
    rng = _rng(seed)
    ns = np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), count)).round().astype(np.int64)
    nxy = rng.integers(box_xy[0], box_xy[1] + 1, count)
    nzs = rng.integers(box_z[0], box_z[1] + 1, count)
    out = []
    for k in range(count):
        dims = (int(nxy[k]), int(nxy[k]), int(nzs[k]))
        n = int(ns[k])
        ell = (dims[0] * dims[1] * dims[2] / n) ** (1.0 / 3.0)
        p = gaussians_uniform((seed, k), n, dims, ls_mean=float(np.log(0.75 * ell)), ls_std=0.3)
        out.append((p, dims))
    return out


def serving_arrivals(seed: int = 5, rate: float = 50.0, duration: float = 120.0, nsets: int = 32,
                     scales=(2.0, 2.5, 3.0, 4.0), fit_fraction: float = 0.1, fit_pool: int = 4):
    """Poisson arrivals at ``rate`` per second over ``duration`` seconds.  Each request is a render
    (probability 1 - fit_fraction: a uniform set and a uniform scale) or a fit (a uniform member
    of a pool of ``fit_pool`` scans).  Returns a list of (t, "render", set_id, scale) and
    (t, "fit", pool_index, None)."""
    rng = _rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        if rng.random() < fit_fraction:
            out.append((t, "fit", int(rng.integers(fit_pool)), None))
        else:
            out.append((t, "render", int(rng.integers(nsets)), float(scales[int(rng.integers(len(scales)))])))


def serving_fit_pool(seed: int = 6, count: int = 4, n_max: int = 200000, f: int = 4, workers: int = 8):
    """Scans for the fit requests of the request loop: uneven-batch grids (batch_dims of a uniform
    index), phantom HR (seed (seed, k)), LR = z-mean of f, Gaussian count exp(U(ln 5e4, ln n_max))
    on the coarsest lattice with enough sites.  Returns a list of (params, lr_obs, dims)."""
    rng = _rng(seed)
    js = rng.integers(0, 16, count)
    ns = np.exp(rng.uniform(np.log(5e4), np.log(n_max), count))

    def one(k):
        dims = batch_dims(int(js[k]))
        lr = zmean_observation(phantom((seed, k), dims), f)
        n = int(min(round(ns[k]), lr.size))
        p = lattice_init((seed, k, 1), lr, n, f, stride_xy=lattice_stride(lr.shape, n))
        return p, lr, dims

    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(one, range(count)))
