"""Oracle: plain, slow, obviously correct CPU reference of the Gaussian-to-voxel renderer.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library and never calls it.

Contents (FP64 unless stated):
  * ``render``, ``render_points``, ``grad``, ``count_pairs``, ``ambiguous``, ``frames``,
    ``index_boxes``: ctypes wrappers over ``oracle.c`` (the rendering equation of §3.2 truncated
    to the 3-sigma ellipsoid of §3.3, and the two gradient equations of §3.3).
  * ``render_bound``, ``grad_bound``: a-priori bounds of this oracle's own rounding error per output
    entry (its FP64 error), from the sums of absolute terms and the term counts.
  * ``render_envelope``: the forward with the inclusion of ambiguous pairs (|d^2 - 9| within a band)
    left open: per voxel the extremes over every include/exclude choice.
  * ``weights_box``: one Gaussian's weights over its index box with the support held fixed (for
    box-local finite differences).
  * ``mse_loss``, ``zmean``, ``zmean_adjoint``, ``fit_l1_loss``, ``l1_sign_ties``: the losses of the
    fit (numpy, FP64) and the LR voxels whose L1 sign a correct FP32 render may take either way.
  * ``adam_step``: Adam with bias correction (numpy), the optimiser of the per-scan fit.
  * ``fit_step``: render -> loss -> gradient -> Adam, composed from the above.

Inputs are the FP32 arrays the GPU path also receives; they are promoted exactly to double.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS: dict = {}

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _lib(long_double: bool = False):
    name = "liboracle_ld.so" if long_double else "liboracle.so"
    if name in _LIBS:
        return _LIBS[name]
    path = os.path.join(_HERE, name)
    if not os.path.exists(path):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(path)
    grid_args = [_int, _int, _int, _f64p, _f64p]
    lib.og_frames.argtypes = [_i64, _f32p, _f32p, _f64p, _f64p, _f64p]
    lib.og_frames.restype = _int
    lib.og_render.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _f64p, _vp, _vp, _int]
    lib.og_render.restype = _int
    lib.og_render_points.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _i64, _i64p,
                                     _f64p, _vp, _vp, _int]
    lib.og_render_points.restype = _int
    lib.og_grad.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _f64p, _f64p, _f64p, _i64,
                            _vp, _f64p, _f64p, _f64p, _f64p, _vp, _int]
    lib.og_grad.restype = _int
    lib.og_count_pairs.argtypes = [_i64, _f32p, _f32p, _f32p, *grid_args, _dbl, _int]
    lib.og_count_pairs.restype = _i64
    lib.og_ambiguous.argtypes = [_i64, _f32p, _f32p, _f32p, *grid_args, _dbl, _dbl, _i64, _vp, _i32p, _int]
    lib.og_ambiguous.restype = _int
    lib.og_index_boxes.argtypes = [_i64, _f32p, _f32p, _f32p, *grid_args, _dbl, _i32p]
    lib.og_index_boxes.restype = _int
    lib.og_render_frozen.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, _f32p, _f32p, _f32p, *grid_args, _dbl,
                                     _dbl, _f64p, _vp, _int]
    lib.og_render_frozen.restype = _int
    lib.og_ambiguous_voxels.argtypes = [_i64, _f32p, _f32p, _f32p, *grid_args, _dbl, _dbl, _i32p, _int]
    lib.og_ambiguous_voxels.restype = _int
    lib.og_render_bound.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _f64p, _f64p,
                                    _f64p, _int]
    lib.og_render_bound.restype = _int
    lib.og_grad_bound.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _f64p, _f64p, _f64p,
                                  _i64, _vp, _f64p, _f64p, _int]
    lib.og_grad_bound.restype = _int
    lib.og_render_envelope.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _vp, *grid_args, _dbl, _dbl, _dbl, _int,
                                       _f64p, _f64p, _f64p, _f64p, _vp, _int]
    lib.og_render_envelope.restype = _i64
    lib.og_weights_box.argtypes = [_f32p, _f32p, _f32p, _f32p, _vp, _f32p, _f32p, _f32p, *grid_args, _dbl, _i32p,
                                   _i64, _vp, _vp]
    lib.og_weights_box.restype = _i64
    _LIBS[name] = lib
    return lib


@dataclass
class Grid:
    """Voxel grid: voxel (ix, iy, iz) has centre origin + spacing * (ix, iy, iz); arrays are
    [nz][ny][nx] (x fastest)."""

    nx: int
    ny: int
    nz: int
    origin: Sequence[float] = (0.5, 0.5, 0.5)
    spacing: Sequence[float] = (1.0, 1.0, 1.0)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def size(self) -> int:
        return self.nx * self.ny * self.nz

    def _args(self):
        return (int(self.nx), int(self.ny), int(self.nz), np.ascontiguousarray(self.origin, dtype=np.float64),
                np.ascontiguousarray(self.spacing, dtype=np.float64))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _params(p: dict):
    n = int(np.asarray(p["amp"]).shape[0])
    mu = _f32(p["mu"]).reshape(n, 3)
    ls = _f32(p["log_scale"]).reshape(n, 3)
    q = _f32(p["quat"]).reshape(n, 4)
    amp = _f32(p["amp"]).reshape(n)
    relax = p.get("relax")
    relax = None if relax is None else _f32(relax).reshape(n)
    return n, mu, ls, q, amp, relax


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def frames(log_scale, quat):
    """R, Sigma, P (each [n,3,3]) of every Gaussian (§3.1: Sigma = R diag(exp(2s)) R^T)."""
    ls = _f32(log_scale).reshape(-1, 3)
    q = _f32(quat).reshape(-1, 4)
    n = ls.shape[0]
    R = np.zeros((n, 9))
    S = np.zeros((n, 9))
    P = np.zeros((n, 9))
    if _lib().og_frames(n, ls, q, R, S, P) != 0:
        raise ValueError("non-finite input or zero quaternion")
    return R.reshape(n, 3, 3), S.reshape(n, 3, 3), P.reshape(n, 3, 3)


def render(p: dict, grid: Grid, cutoff: float = 3.0, eps: float = 1e-8, threads: Optional[int] = None,
           long_double: bool = False):
    """Forward render on the whole grid.  Returns (I, W, S), each float64 [nz, ny, nx]."""
    n, mu, ls, q, amp, relax = _params(p)
    I = np.zeros(grid.size)
    W = np.zeros(grid.size)
    S = np.zeros(grid.size)
    rc = _lib(long_double).og_render(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps), I,
                                     _ptr(W), _ptr(S), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle render failed ({rc}): non-finite input or zero quaternion")
    return I.reshape(grid.shape), W.reshape(grid.shape), S.reshape(grid.shape)


def render_frozen(p: dict, support: dict, grid: Grid, cutoff: float = 3.0, eps: float = 1e-8,
                  threads: Optional[int] = None):
    """Forward whose pair predicate uses the positions, scales and rotations of ``support`` and whose
    weights use those of ``p`` (the support held fixed, for finite differences).  Returns (I, W)."""
    n, mu, ls, q, amp, relax = _params(p)
    _, mu0, ls0, q0, _, _ = _params(support)
    I = np.zeros(grid.size)
    W = np.zeros(grid.size)
    rc = _lib().og_render_frozen(n, mu, ls, q, amp, _ptr(relax), mu0, ls0, q0, *grid._args(), float(cutoff),
                                 float(eps), I, _ptr(W), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle render_frozen failed ({rc})")
    return I.reshape(grid.shape), W.reshape(grid.shape)


def render_points(p: dict, grid: Grid, vox, cutoff: float = 3.0, eps: float = 1e-8, threads: Optional[int] = None):
    """Forward at the given flat voxel indices.  Returns (I, W, S) float64 [len(vox)]."""
    n, mu, ls, q, amp, relax = _params(p)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    m = vox.shape[0]
    I = np.zeros(m)
    W = np.zeros(m)
    S = np.zeros(m)
    rc = _lib().og_render_points(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps), m, vox,
                                 I, _ptr(W), _ptr(S), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle render_points failed ({rc})")
    return I, W, S


def grad(p: dict, grid: Grid, I, W, gI, cutoff: float = 3.0, eps: float = 1e-8, sel=None,
         threads: Optional[int] = None, long_double: bool = False):
    """Gradients of L w.r.t. (mu, log_scale, quat, amp, relax) given the forward's I, W and dL/dI.

    ``sel``: optional Gaussian indices; the returned arrays are n-sized and only the selected rows
    are meaningful (others are NaN)."""
    n, mu, ls, q, amp, relax = _params(p)
    I = np.ascontiguousarray(I, dtype=np.float64).reshape(-1)
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
    gI = np.ascontiguousarray(gI, dtype=np.float64).reshape(-1)
    assert I.size == W.size == gI.size == grid.size
    out = {k: np.full(s, np.nan) for k, s in
           (("mu", (n, 3)), ("log_scale", (n, 3)), ("quat", (n, 4)), ("amp", (n,)), ("relax", (n,)))}
    selv = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    rc = _lib(long_double).og_grad(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps), I, W,
                                   gI, 0 if selv is None else selv.shape[0], _ptr(selv), out["mu"], out["log_scale"],
                                   out["quat"], out["amp"], _ptr(out["relax"]), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle grad failed ({rc})")
    return out


def count_pairs(p: dict, grid: Grid, cutoff: float = 3.0, threads: Optional[int] = None) -> int:
    """Number of useful (voxel, Gaussian) pairs: d^2 <= cutoff^2."""
    n, mu, ls, q, _, _ = _params(p)
    c = _lib().og_count_pairs(n, mu, ls, q, *grid._args(), float(cutoff), threads or default_threads())
    if c < 0:
        raise ValueError("oracle count_pairs failed")
    return int(c)


def ambiguous(p: dict, grid: Grid, band: float, cutoff: float = 3.0, sel=None, threads: Optional[int] = None):
    """Per (selected) Gaussian: number of voxels with |d^2 - cutoff^2| <= band."""
    n, mu, ls, q, _, _ = _params(p)
    selv = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    m = n if selv is None else selv.shape[0]
    cnt = np.zeros(m, dtype=np.int32)
    rc = _lib().og_ambiguous(n, mu, ls, q, *grid._args(), float(cutoff), float(band), 0 if selv is None else m,
                             _ptr(selv), cnt, threads or default_threads())
    if rc != 0:
        raise ValueError("oracle ambiguous failed")
    return cnt


def ambiguous_voxels(p: dict, grid: Grid, band: float, cutoff: float = 3.0, threads: Optional[int] = None):
    """Per voxel [nz, ny, nx]: number of Gaussians with |d^2 - cutoff^2| <= band there."""
    n, mu, ls, q, _, _ = _params(p)
    cnt = np.zeros(grid.size, dtype=np.int32)
    if _lib().og_ambiguous_voxels(n, mu, ls, q, *grid._args(), float(cutoff), float(band), cnt,
                                  threads or default_threads()) != 0:
        raise ValueError("oracle ambiguous_voxels failed")
    return cnt.reshape(grid.shape)


def index_boxes(p: dict, grid: Grid, cutoff: float = 3.0):
    """Inclusive voxel index box [n, 6] = (lo x, y, z, hi x, y, z) of each Gaussian's padded
    3-sigma axis-aligned box."""
    n, mu, ls, q, _, _ = _params(p)
    box = np.zeros((n, 6), dtype=np.int32)
    if _lib().og_index_boxes(n, mu, ls, q, *grid._args(), float(cutoff), box) != 0:
        raise ValueError("oracle index_boxes failed")
    return box


def render_bound(p: dict, grid: Grid, cutoff: float = 3.0, eps: float = 1e-8, threads: Optional[int] = None,
                 long_double: bool = False):
    """A-priori bound of this oracle's rounding error in ``render``: per voxel |I_computed - I_exact|
    <= bI and likewise bW (arrays [nz, ny, nx]), valid when every pair is decided as exact
    arithmetic decides it, i.e. when the returned margin (the smallest |d^2 - cutoff^2| minus that
    pair's d^2 error bound over all visited pairs) is positive.  Returns (bI, bW, margin)."""
    n, mu, ls, q, amp, relax = _params(p)
    bI = np.zeros(grid.size)
    bW = np.zeros(grid.size)
    margin = np.zeros(1)
    rc = _lib(long_double).og_render_bound(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps),
                                           bI, bW, margin, threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle render_bound failed ({rc})")
    return bI.reshape(grid.shape), bW.reshape(grid.shape), float(margin[0])


def grad_bound(p: dict, grid: Grid, I, W, gI, cutoff: float = 3.0, eps: float = 1e-8, sel=None,
               threads: Optional[int] = None, long_double: bool = False):
    """A-priori bound of this oracle's rounding error in ``grad`` (same arguments): a dict of arrays
    shaped like ``grad``'s outputs (rows not selected are NaN), and the margin as in
    ``render_bound``."""
    n, mu, ls, q, amp, relax = _params(p)
    I = np.ascontiguousarray(I, dtype=np.float64).reshape(-1)
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1)
    gI = np.ascontiguousarray(gI, dtype=np.float64).reshape(-1)
    assert I.size == W.size == gI.size == grid.size
    b = np.full((n, 12), np.nan)
    margin = np.zeros(1)
    selv = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    rc = _lib(long_double).og_grad_bound(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps), I,
                                         W, gI, 0 if selv is None else selv.shape[0], _ptr(selv), b, margin,
                                         threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle grad_bound failed ({rc})")
    out = {"mu": b[:, 0:3], "log_scale": b[:, 3:6], "quat": b[:, 6:10], "amp": b[:, 10], "relax": b[:, 11]}
    return {k: np.ascontiguousarray(v) for k, v in out.items()}, float(margin[0])


def render_envelope(p: dict, grid: Grid, band: float, cutoff: float = 3.0, eps: float = 1e-8, maxk: int = 12,
                    threads: Optional[int] = None):
    """Forward with every ambiguous pair (|d^2 - cutoff^2| <= band) free to be included or not.
    Returns (Ilo, Ihi, Wlo, Whi, namb, skipped): per voxel the extremes of I and W over all
    include/exclude choices of its namb ambiguous pairs (lo = hi = the forward where namb = 0;
    -inf / +inf where namb > maxk, counted in skipped)."""
    n, mu, ls, q, amp, relax = _params(p)
    Ilo, Ihi, Wlo, Whi = (np.zeros(grid.size) for _ in range(4))
    namb = np.zeros(grid.size, dtype=np.int32)
    sk = _lib().og_render_envelope(n, mu, ls, q, amp, _ptr(relax), *grid._args(), float(cutoff), float(eps),
                                   float(band), int(maxk), Ilo, Ihi, Wlo, Whi, _ptr(namb),
                                   threads or default_threads())
    if sk < 0:
        raise ValueError(f"oracle render_envelope failed ({sk})")
    sh = grid.shape
    return Ilo.reshape(sh), Ihi.reshape(sh), Wlo.reshape(sh), Whi.reshape(sh), namb.reshape(sh), int(sk)


def weights_box(p: dict, j: int, grid: Grid, support: Optional[dict] = None, cutoff: float = 3.0):
    """Weights of Gaussian j of ``p`` over the padded index box of Gaussian j of ``support`` (default
    ``p``), with the pair predicate taken from ``support`` (the support held fixed).  Returns
    (flat voxel indices int64, weights float64); pairs outside the support weigh 0."""
    support = p if support is None else support

    def one(d, keys):
        return [_f32(d[k]).reshape(np.asarray(d[k]).shape[0], -1)[j].copy() for k in keys]

    mu, ls, q, amp = one(p, ("mu", "log_scale", "quat", "amp"))
    relax = None if p.get("relax") is None else _f32(p["relax"]).reshape(-1)[j:j + 1].copy()
    mu0, ls0, q0 = one(support, ("mu", "log_scale", "quat"))
    box = np.zeros(6, dtype=np.int32)
    lib = _lib()
    cnt = lib.og_weights_box(mu, ls, q, amp, _ptr(relax), mu0, ls0, q0, *grid._args(), float(cutoff), box, 0, None,
                             None)
    if cnt < 0:
        raise ValueError("oracle weights_box: invalid Gaussian")
    vox = np.zeros(cnt, dtype=np.int64)
    w = np.zeros(cnt)
    if cnt:
        lib.og_weights_box(mu, ls, q, amp, _ptr(relax), mu0, ls0, q0, *grid._args(), float(cutoff), box, cnt,
                           _ptr(vox), _ptr(w))
    return vox, w


# ------------------------------------------------------------------------------------------------
# Losses of the fit (numpy, FP64).


def mse_loss(I, T):
    """L = mean((I - T)^2); returns (L, dL/dI)."""
    I = np.asarray(I, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    d = I - T
    return float(np.mean(d * d)), 2.0 * d / d.size


def zmean(I, f: int = 4):
    """Mean of f consecutive z slices: [nz, ny, nx] -> [nz/f, ny, nx]."""
    I = np.asarray(I, dtype=np.float64)
    nz, ny, nx = I.shape
    assert nz % f == 0
    return I.reshape(nz // f, f, ny, nx).mean(axis=1)


def zmean_adjoint(G, f: int = 4):
    """Adjoint of ``zmean``: each HR voxel receives its LR voxel's value / f."""
    G = np.asarray(G, dtype=np.float64)
    return np.repeat(G, f, axis=0) / f


def fit_l1_loss(I, O, f: int = 4):
    """Fit loss: L = mean |zmean(I) - O| over LR voxels; returns (L, dL/dI at HR), with
    dL/dI = sign(zmean(I) - O) / (f * nLR) on the f HR voxels of each LR voxel and sign(0) = 0, all
    in FP64."""
    LR = zmean(I, f)
    d = LR - np.asarray(O, dtype=np.float64)
    L = float(np.mean(np.abs(d)))
    return L, zmean_adjoint(np.sign(d) / d.size, f)


# An FP32 render that meets the forward tolerance (|I - I_exact| <= FWD_RTOL |I| + FWD_ATOL per
# voxel) has a z-mean within FWD_RTOL max|I| + FWD_ATOL of the exact one, plus the FP32 rounding of
# the f-term sum and its scaling (at most (f + 1) 2^-24 of the sum of |I|).
FWD_RTOL, FWD_ATOL = 1e-5, 1e-7


def l1_sign_band(I, f: int = 4):
    """Per LR voxel [nz/f, ny, nx]: how far a render meeting the forward tolerance may put its
    z-mean from this one, FWD_RTOL max_j |I_j| + FWD_ATOL + (f + 1) 2^-24 sum_j |I_j| / f over the
    LR voxel's f HR voxels j."""
    I = np.asarray(I, dtype=np.float64)
    nz, ny, nx = I.shape
    g = np.abs(I).reshape(nz // f, f, ny, nx)
    return FWD_RTOL * g.max(axis=1) + FWD_ATOL + (f + 1) * 2.0 ** -24 * g.sum(axis=1) / f


def l1_sign_ties(I, O, f: int = 4):
    """LR voxels where |zmean(I) - O| is within ``l1_sign_band``: there either sign (and 0) of the
    L1 gradient is a correct result."""
    return np.abs(zmean(I, f) - np.asarray(O, dtype=np.float64)) <= l1_sign_band(I, f)


# ------------------------------------------------------------------------------------------------
# Adam (numpy, FP64).  Parameter groups in order: mu, log_scale, quat, amp, relax.

GROUPS = ("mu", "log_scale", "quat", "amp", "relax")


def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int, lr: dict, beta1=0.9, beta2=0.999,
              eps=1e-8):
    """One Adam step with bias correction (step counts from 1).  Returns new (params, m, v), all
    float64; groups with lr == 0 keep their values (their moments still update)."""
    newp, newm, newv = {}, {}, {}
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    for k in GROUPS:
        g = np.asarray(grads[k], dtype=np.float64)
        mk = beta1 * np.asarray(m[k], dtype=np.float64) + (1.0 - beta1) * g
        vk = beta2 * np.asarray(v[k], dtype=np.float64) + (1.0 - beta2) * g * g
        mhat = mk / bc1
        vhat = vk / bc2
        newp[k] = np.asarray(params[k], dtype=np.float64) - lr[k] * mhat / (np.sqrt(vhat) + eps)
        newm[k], newv[k] = mk, vk
    return newp, newm, newv


def fit_step(params: dict, O, grid: Grid, m: dict, v: dict, step: int, lr: dict, cutoff=3.0, eps=1e-8, f=4,
             beta1=0.9, beta2=0.999, adam_eps=1e-8, threads=None):
    """One step of the per-scan fit: render -> z-mean-of-f -> L1 -> gradient -> Adam.

    Returns (loss, new_params (float64), new_m, new_v, grads)."""
    I, W, _ = render(params, grid, cutoff, eps, threads)
    L, gI = fit_l1_loss(I, O, f)
    gr = grad(params, grid, I, W, gI, cutoff, eps, threads=threads)
    newp, newm, newv = adam_step(params, gr, m, v, step, lr, beta1, beta2, adam_eps)
    return L, newp, newm, newv, gr
