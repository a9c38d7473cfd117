"""Python binding of libgs.so (include/gs.h): ctypes marshalling of torch device tensors.

Every computation runs in the library's HIP kernels; this module only builds the C structs, takes
device pointers from torch tensors and passes torch's current HIP stream.  Importing it fails
loudly if the library has not been built (there is no fallback path).

The ``gs_*`` functions mirror the C entry points one to one.  ``Bins``, ``render``, ``backward``
and ``FitState`` are conveniences that size and allocate the caller-owned buffers with torch.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_2603_09621_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

GS_STATIC_SCRATCH_BYTES = 64 << 20  # the header's GS_STATIC_SCRATCH_BYTES
GS_OK, GS_ERR_INVALID_ARG, GS_ERR_CAPACITY, GS_ERR_NONFINITE, GS_ERR_HIP, GS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
_ERR_NAMES = {-1: "INVALID_ARG", -2: "CAPACITY", -3: "NONFINITE", -4: "HIP", -5: "UNSUPPORTED"}


class GSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"GS_ERR_{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class CapacityError(GSError):
    pass


_vp = ctypes.c_void_p
_fp = ctypes.POINTER(ctypes.c_float)


class gs_gaussians_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mu", _vp), ("log_scale", _vp), ("quat", _vp), ("amp", _vp), ("relax", _vp)]


class gs_grid_t(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3)]


class gs_opts_t(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32), ("cutoff", ctypes.c_float),
                ("eps", ctypes.c_float), ("flags", ctypes.c_uint32)]


class gs_bins_t(ctypes.Structure):
    _fields_ = [("ws", _vp), ("ws_bytes", ctypes.c_size_t), ("key_capacity", ctypes.c_int64)]


class gs_grads_t(ctypes.Structure):
    _fields_ = [("d_mu", _vp), ("d_log_scale", _vp), ("d_quat", _vp), ("d_amp", _vp), ("d_relax", _vp)]


class gs_adam_t(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 5), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class gs_fit_state_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mu", _vp), ("log_scale", _vp), ("quat", _vp), ("amp", _vp), ("relax", _vp),
                ("m", _vp), ("v", _vp), ("step", _vp)]


class gs_fit_opts_t(ctypes.Structure):
    _fields_ = [("hr", gs_grid_t), ("opts", gs_opts_t), ("zdown", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("adam", gs_adam_t)]


class gs_fit_buffers_t(ctypes.Structure):
    _fields_ = [("I", _vp), ("W", _vp), ("dL_dI", _vp), ("grads", gs_grads_t), ("scratch", _vp),
                ("scratch_bytes", ctypes.c_size_t), ("loss", _vp)]


class gs_batch_t(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int32), ("n", ctypes.POINTER(ctypes.c_int64)), ("grid", ctypes.POINTER(gs_grid_t)),
                ("sets", ctypes.POINTER(gs_gaussians_t))]


class gs_status_t(ctypes.Structure):
    _fields_ = [("n_keys", ctypes.c_int64), ("overflow", ctypes.c_int32), ("nonfinite", ctypes.c_int32)]


_P = ctypes.POINTER
_sigs = {
    "gs_workspace_size": [ctypes.c_int64, _P(gs_grid_t), _P(gs_opts_t), ctypes.c_int64, _P(ctypes.c_size_t)],
    "gs_brick_supported": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "gs_bin_query": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _P(ctypes.c_int64)],
    "gs_bin": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp],
    "gs_render_fwd": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp, _vp],
    "gs_count_pairs": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp],
    "gs_count_evals": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp],
    "gs_render_bwd": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp, _vp,
                      _P(gs_grads_t), _vp],
    "gs_loss_mse": [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_size_t, _vp],
    "gs_loss_l1_zmean": [_vp, _vp, _P(gs_grid_t), ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t, _vp],
    "gs_adam_step": [_P(gs_fit_state_t), _P(gs_grads_t), _P(gs_adam_t), _P(gs_bins_t), _vp],
    "gs_fit_step": [_P(gs_fit_state_t), _vp, _P(gs_fit_opts_t), _P(gs_bins_t), _P(gs_fit_buffers_t), _vp],
    "gs_status": [_P(gs_bins_t), _vp, _P(gs_status_t)],
    "gs_render_fwd_noalloc": [_P(gs_gaussians_t), _P(gs_grid_t), _P(gs_opts_t), _vp, _vp, _vp, _vp],
    "gs_workspace_size_batch": [_P(gs_batch_t), _P(gs_opts_t), ctypes.c_int64, _P(ctypes.c_size_t)],
    "gs_bin_query_batch": [_P(gs_gaussians_t), _P(gs_batch_t), _P(gs_opts_t), _P(gs_bins_t), _vp,
                           _P(ctypes.c_int64)],
    "gs_bin_batch": [_P(gs_gaussians_t), _P(gs_batch_t), _P(gs_opts_t), _P(gs_bins_t), _vp],
    "gs_render_fwd_batch": [_P(gs_gaussians_t), _P(gs_batch_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp, _vp],
    "gs_count_pairs_batch": [_P(gs_gaussians_t), _P(gs_batch_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp],
    "gs_render_bwd_batch": [_P(gs_gaussians_t), _P(gs_batch_t), _P(gs_opts_t), _P(gs_bins_t), _vp, _vp, _vp,
                            _P(gs_grads_t), _vp],
    "gs_fit_step_batch": [_P(gs_fit_state_t), _vp, _P(gs_batch_t), _P(gs_fit_opts_t), _P(gs_bins_t),
                          _P(gs_fit_buffers_t), _vp],
    "gs_profile_enable": [ctypes.c_int],
    "gs_profile_reset": [],
    "gs_profile_read": [_vp, ctypes.c_int, _vp, _P(ctypes.c_int64), _P(ctypes.c_double), _P(ctypes.c_int)],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.gs_loss_scratch_bytes.argtypes = [ctypes.c_int64]
_lib.gs_loss_scratch_bytes.restype = ctypes.c_size_t
_lib.gs_fit_scratch_bytes.argtypes = [_P(gs_grid_t)]
_lib.gs_fit_scratch_bytes.restype = ctypes.c_size_t
_lib.gs_fit_scratch_bytes_batch.argtypes = [_P(gs_batch_t)]
_lib.gs_fit_scratch_bytes_batch.restype = ctypes.c_size_t
_lib.gs_last_error.argtypes = []
_lib.gs_last_error.restype = ctypes.c_char_p

EXPORTED = tuple(_sigs) + ("gs_loss_scratch_bytes", "gs_fit_scratch_bytes", "gs_fit_scratch_bytes_batch",
                           "gs_last_error")
MAX_SCANS = 16


def gs_last_error() -> str:
    return _lib.gs_last_error().decode()


def _check(rc: int):
    if rc != GS_OK:
        msg = gs_last_error()
        if rc == GS_ERR_CAPACITY:
            raise CapacityError(rc, msg)
        raise GSError(rc, msg)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t: Optional[torch.Tensor]) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if t.dtype != torch.float32:
        raise ValueError(f"float32 tensor expected, got {t.dtype}")
    return t


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------------------------------------
# Plain-data descriptions


@dataclass
class Grid:
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

    def c(self) -> gs_grid_t:
        return gs_grid_t(self.nx, self.ny, self.nz, (ctypes.c_float * 3)(*self.origin),
                         (ctypes.c_float * 3)(*self.spacing))

    @staticmethod
    def at_scale(lr_dims, scale: float) -> "Grid":
        """Grid of round(scale * dims) voxels covering the same extent as an LR grid of unit spacing
        and origin 0.5 (cell-centred; rendering at an arbitrary scale)."""
        nx, ny, nz = (int(round(scale * d)) for d in lr_dims)
        sp = tuple(d / n for d, n in zip(lr_dims, (nx, ny, nz)))
        return Grid(nx, ny, nz, tuple(0.5 * s for s in sp), sp)


FLAG_FORWARD_ONLY = 1
# tuning bits (speed only; results are bitwise the same)
FLAG_BWD_ONE_BRICK = 1 << 4
FLAG_BWD_WINDOW_256 = 1 << 5
FLAG_BWD_TWO_BRICKS = 1 << 8
FLAG_EMIT_STAGE_4K = 1 << 6
FLAG_EMIT_STAGE_6K = 1 << 7


@dataclass
class Opts:
    bx: int = 8
    by: int = 8
    bz: int = 4
    cutoff: float = 3.0
    eps: float = 1e-8
    forward_only: bool = False  # workspace without the backward's partial sums
    # tuning (speed only): bricks per backward workgroup (8: eight waves; 2 or 1: one wave), the
    # backward's ordering window (512: the default size, 2048 keys for eight bricks and 512 for one or
    # two; 256: half of it), the emit's LDS stage (0: chosen from the key capacity, else 4096 or 6144
    # keys)
    bwd_bricks: int = 8
    bwd_window: int = 512
    emit_stage: int = 0

    @property
    def flags(self) -> int:
        if self.bwd_bricks not in (1, 2, 8) or self.bwd_window not in (256, 512) or self.emit_stage not in (0, 4096, 6144):
            raise ValueError(f"unsupported tuning {self.tuning}")
        f = FLAG_FORWARD_ONLY if self.forward_only else 0
        f |= {1: FLAG_BWD_ONE_BRICK, 2: FLAG_BWD_TWO_BRICKS, 8: 0}[self.bwd_bricks]
        f |= FLAG_BWD_WINDOW_256 if self.bwd_window == 256 else 0
        f |= {0: 0, 4096: FLAG_EMIT_STAGE_4K, 6144: FLAG_EMIT_STAGE_6K}[self.emit_stage]
        return f

    @property
    def tuning(self) -> dict:
        return {"bx": self.bx, "bwd_bricks": self.bwd_bricks, "bwd_window": self.bwd_window,
                "emit_stage": self.emit_stage}

    def with_(self, **kw) -> "Opts":
        return replace(self, **kw)

    def c(self) -> gs_opts_t:
        return gs_opts_t(self.bx, self.by, self.bz, self.cutoff, self.eps, self.flags)


GROUPS = ("mu", "log_scale", "quat", "amp", "relax")


class Batch:
    """Scans handled by the same launches: Gaussian counts and grids, in concatenation order.  With
    ``sets`` (one Gaussians per scan) the bin/render/count calls read every scan's own tensors and
    take ``g=None``."""

    def __init__(self, ns: Sequence[int], grids: Sequence[Grid], sets: Optional[Sequence["Gaussians"]] = None):
        if len(ns) != len(grids) or (sets is not None and len(sets) != len(ns)):
            raise ValueError("one Gaussian count (and set) per grid expected")
        self.ns = [int(n) for n in ns]
        self.grids = list(grids)
        self.sets = None if sets is None else list(sets)

    @staticmethod
    def of_sets(sets: Sequence["Gaussians"], grids: Sequence[Grid]) -> "Batch":
        return Batch([s.n for s in sets], grids, sets)

    def __len__(self) -> int:
        return len(self.ns)

    @property
    def n_total(self) -> int:
        return sum(self.ns)

    @property
    def g_offsets(self):
        return [sum(self.ns[:k]) for k in range(len(self.ns) + 1)]

    @property
    def v_offsets(self):
        return [sum(g.size for g in self.grids[:k]) for k in range(len(self.grids) + 1)]

    def lr_offsets(self, zdown: int):
        return [sum(g.size // zdown for g in self.grids[:k]) for k in range(len(self.grids) + 1)]

    def split(self, flat: torch.Tensor):
        """Per-scan [nz, ny, nx] views of a concatenated volume."""
        o = self.v_offsets
        return [flat[o[k]:o[k + 1]].view(g.shape) for k, g in enumerate(self.grids)]

    def c(self) -> gs_batch_t:
        narr = (ctypes.c_int64 * len(self.ns))(*self.ns)
        garr = (gs_grid_t * len(self.grids))(*[g.c() for g in self.grids])
        sarr = None
        if self.sets is not None:
            sarr = (gs_gaussians_t * len(self.sets))(*[x.c() for x in self.sets])
        b = gs_batch_t(len(self.ns), narr, garr, sarr)
        b._keep = (narr, garr, sarr)  # the arrays must outlive the call
        return b


@dataclass
class Gaussians:
    """Device tensors of one Gaussian set (float32, contiguous)."""

    mu: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    amp: torch.Tensor
    relax: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.amp.shape[0])

    @staticmethod
    def from_numpy(p: dict, device="cuda") -> "Gaussians":
        def t(k):
            v = p.get(k)
            return None if v is None else torch.as_tensor(v, dtype=torch.float32).contiguous().to(device)

        return Gaussians(t("mu"), t("log_scale"), t("quat"), t("amp"), t("relax"))

    def c(self) -> gs_gaussians_t:
        return gs_gaussians_t(self.n, _ptr(_f32(self.mu)), _ptr(_f32(self.log_scale)), _ptr(_f32(self.quat)),
                              _ptr(_f32(self.amp)), _ptr(_f32(self.relax)))


def brick_supported(bx: int, by: int, bz: int) -> bool:
    return bool(_lib.gs_brick_supported(bx, by, bz))


def gs_workspace_size(n: int, grid: Grid, opts: Opts, key_capacity: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.gs_workspace_size(n, ctypes.byref(grid.c()), ctypes.byref(opts.c()), key_capacity,
                                  ctypes.byref(out)))
    return int(out.value)


def gs_loss_scratch_bytes(nvox: int) -> int:
    return int(_lib.gs_loss_scratch_bytes(nvox))


def gs_fit_scratch_bytes(grid: "Grid") -> int:
    return int(_lib.gs_fit_scratch_bytes(ctypes.byref(grid.c())))


def gs_workspace_size_batch(batch: Batch, opts: Opts, key_capacity: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.gs_workspace_size_batch(ctypes.byref(batch.c()), ctypes.byref(opts.c()), key_capacity,
                                        ctypes.byref(out)))
    return int(out.value)


def gs_fit_scratch_bytes_batch(batch: Batch) -> int:
    return int(_lib.gs_fit_scratch_bytes_batch(ctypes.byref(batch.c())))


class Bins:
    """Caller-owned binning workspace (a uint8 device tensor) for one Gaussian count and grid, or
    for a batch of scans (``grid`` a Batch; ``n`` is then ignored)."""

    def __init__(self, n: int, grid, opts: Opts, key_capacity: int, device="cuda"):
        self.grid, self.opts, self.key_capacity = grid, opts, int(key_capacity)
        if isinstance(grid, Batch):
            self.n = grid.n_total
            self.ws_bytes = gs_workspace_size_batch(grid, opts, self.key_capacity)
        else:
            self.n = n
            self.ws_bytes = gs_workspace_size(n, grid, opts, self.key_capacity)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def c(self) -> gs_bins_t:
        return gs_bins_t(ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.key_capacity)


def gs_bin_query(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check(_lib.gs_bin_query(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                             ctypes.byref(bins.c()), _stream(stream), ctypes.byref(out)))
    return int(out.value)


def gs_bin(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, stream=None) -> None:
    _check(_lib.gs_bin(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()), ctypes.byref(bins.c()),
                       _stream(stream)))


def gs_render_fwd(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, I: torch.Tensor, W: Optional[torch.Tensor] = None,
                  stream=None) -> None:
    _check(_lib.gs_render_fwd(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                              ctypes.byref(bins.c()), _ptr(_f32(I)), _ptr(_f32(W)), _stream(stream)))


EVAL_COUNTS = ("useful_pairs", "fwd_evals", "fwd_issued", "bwd_evals", "bwd_issued", "bwd_box_rows")


def gs_count_evals(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, out: torch.Tensor, stream=None) -> None:
    """The six evaluation counts (``EVAL_COUNTS``) into a device int64 tensor of 6 entries."""
    if out.dtype != torch.int64 or out.numel() < len(EVAL_COUNTS) or not out.is_contiguous():
        raise ValueError("contiguous int64 tensor of 6 entries expected")
    _check(_lib.gs_count_evals(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                               ctypes.byref(bins.c()), _ptr(out), _stream(stream)))


def gs_render_fwd_noalloc(g: Gaussians, grid: Grid, opts: Opts, I: torch.Tensor, W: Optional[torch.Tensor] = None,
                          status: Optional[torch.Tensor] = None, stream=None) -> None:
    """Bin + forward with the binning workspace in the library's static device scratch.  status: an
    optional device int64 tensor of 2 entries receiving the gs_status_t block (n_keys, then overflow
    and nonfinite as two int32 in the second entry)."""
    if status is not None and (status.dtype != torch.int64 or status.numel() < 2 or not status.is_contiguous()):
        raise ValueError("status must be a contiguous int64 tensor of at least 2 entries")
    _check(_lib.gs_render_fwd_noalloc(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                                      _ptr(_f32(I)), _ptr(_f32(W)), _ptr(status), _stream(stream)))


def unpack_status(status: torch.Tensor) -> dict:
    """The gs_status_t block written by gs_render_fwd_noalloc, read back to the host."""
    v = status[:2].cpu()
    flags = int(v[1])
    return {"n_keys": int(v[0]), "overflow": flags & 0xFFFFFFFF, "nonfinite": (flags >> 32) & 0xFFFFFFFF}


def gs_count_pairs(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, out: torch.Tensor, stream=None) -> None:
    if out.dtype != torch.int64:
        raise ValueError("int64 tensor expected")
    _check(_lib.gs_count_pairs(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                               ctypes.byref(bins.c()), _ptr(out), _stream(stream)))


@dataclass
class Grads:
    mu: torch.Tensor
    log_scale: torch.Tensor
    quat: torch.Tensor
    amp: torch.Tensor
    relax: Optional[torch.Tensor] = None

    @staticmethod
    def empty(n: int, relax: bool = True, device="cuda") -> "Grads":
        z = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)  # noqa: E731
        return Grads(z(n, 3), z(n, 3), z(n, 4), z(n), z(n) if relax else None)

    def c(self) -> gs_grads_t:
        return gs_grads_t(_ptr(self.mu), _ptr(self.log_scale), _ptr(self.quat), _ptr(self.amp), _ptr(self.relax))

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in GROUPS}


def gs_render_bwd(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, I: torch.Tensor, W: torch.Tensor,
                  dL_dI: torch.Tensor, grads: Grads, stream=None) -> None:
    _check(_lib.gs_render_bwd(ctypes.byref(g.c()), ctypes.byref(grid.c()), ctypes.byref(opts.c()),
                              ctypes.byref(bins.c()), _ptr(_f32(I)), _ptr(_f32(W)), _ptr(_f32(dL_dI)),
                              ctypes.byref(grads.c()), _stream(stream)))


def gs_loss_mse(I: torch.Tensor, T: torch.Tensor, dL_dI: torch.Tensor, loss: torch.Tensor, scratch: torch.Tensor,
                stream=None) -> None:
    _check(_lib.gs_loss_mse(_ptr(_f32(I)), _ptr(_f32(T)), I.numel(), _ptr(_f32(dL_dI)), _ptr(_f32(loss)),
                            _ptr(scratch), scratch.numel() * scratch.element_size(), _stream(stream)))


def gs_loss_l1_zmean(I: torch.Tensor, obs: torch.Tensor, grid: Grid, zdown: int, dL_dI: torch.Tensor,
                     loss: torch.Tensor, scratch: torch.Tensor, stream=None) -> None:
    _check(_lib.gs_loss_l1_zmean(_ptr(_f32(I)), _ptr(_f32(obs)), ctypes.byref(grid.c()), zdown, _ptr(_f32(dL_dI)),
                                 _ptr(_f32(loss)), _ptr(scratch), scratch.numel() * scratch.element_size(),
                                 _stream(stream)))


def _gptr(g: Optional["Gaussians"]):
    return None if g is None else ctypes.byref(g.c())


def gs_bin_query_batch(g: Gaussians, batch: Batch, opts: Opts, bins: Bins, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check(_lib.gs_bin_query_batch(_gptr(g), ctypes.byref(batch.c()), ctypes.byref(opts.c()),
                                   ctypes.byref(bins.c()), _stream(stream), ctypes.byref(out)))
    return int(out.value)


def gs_bin_batch(g: Gaussians, batch: Batch, opts: Opts, bins: Bins, stream=None) -> None:
    _check(_lib.gs_bin_batch(_gptr(g), ctypes.byref(batch.c()), ctypes.byref(opts.c()),
                             ctypes.byref(bins.c()), _stream(stream)))


def gs_render_fwd_batch(g: Gaussians, batch: Batch, opts: Opts, bins: Bins, I: torch.Tensor,
                        W: Optional[torch.Tensor] = None, stream=None) -> None:
    _check(_lib.gs_render_fwd_batch(_gptr(g), ctypes.byref(batch.c()), ctypes.byref(opts.c()),
                                    ctypes.byref(bins.c()), _ptr(_f32(I)), _ptr(_f32(W)), _stream(stream)))


def gs_count_pairs_batch(g: Gaussians, batch: Batch, opts: Opts, bins: Bins, out: torch.Tensor, stream=None) -> None:
    if out.dtype != torch.int64:
        raise ValueError("int64 tensor expected")
    _check(_lib.gs_count_pairs_batch(_gptr(g), ctypes.byref(batch.c()), ctypes.byref(opts.c()),
                                     ctypes.byref(bins.c()), _ptr(out), _stream(stream)))


def gs_render_bwd_batch(g: Gaussians, batch: Batch, opts: Opts, bins: Bins, I: torch.Tensor, W: torch.Tensor,
                        dL_dI: torch.Tensor, grads: "Grads", stream=None) -> None:
    _check(_lib.gs_render_bwd_batch(ctypes.byref(g.c()), ctypes.byref(batch.c()), ctypes.byref(opts.c()),
                                    ctypes.byref(bins.c()), _ptr(_f32(I)), _ptr(_f32(W)), _ptr(_f32(dL_dI)),
                                    ctypes.byref(grads.c()), _stream(stream)))


def gs_status(bins: Bins, stream=None, raise_on_error: bool = True):
    st = gs_status_t()
    rc = _lib.gs_status(ctypes.byref(bins.c()), _stream(stream), ctypes.byref(st))
    if raise_on_error:
        _check(rc)
    return {"rc": rc, "n_keys": int(st.n_keys), "overflow": int(st.overflow), "nonfinite": int(st.nonfinite)}


# ------------------------------------------------------------------------------------------------
# Profiling


def profile_enable(on: bool = True) -> None:
    _check(_lib.gs_profile_enable(1 if on else 0))


def profile_reset() -> None:
    _check(_lib.gs_profile_reset())


def profile_read(stream=None) -> dict:
    cap = 64
    names = (ctypes.c_char * 48 * cap)()
    launches = (ctypes.c_int64 * cap)()
    total = (ctypes.c_double * cap)()
    n = ctypes.c_int(0)
    _check(_lib.gs_profile_read(_stream(stream), cap, ctypes.cast(names, _vp), launches, total, ctypes.byref(n)))
    out = {}
    for i in range(n.value):
        out[bytes(names[i]).split(b"\0", 1)[0].decode()] = (int(launches[i]), float(total[i]))
    return out


# ------------------------------------------------------------------------------------------------
# Conveniences


def plan_bins(g: Gaussians, grid: Grid, opts: Opts, headroom: float = 1.25, min_capacity: int = 1024,
              stream=None) -> Bins:
    """Workspace with room for the exact key count of ``g`` times ``headroom`` (one synchronising
    count pass)."""
    probe = Bins(g.n, grid, opts, 0, device=g.amp.device if g.n else "cuda")
    k = gs_bin_query(g, grid, opts, probe, stream)
    return Bins(g.n, grid, opts, max(min_capacity, int(math.ceil(k * headroom))), device=probe.ws.device)


def plan_bins_batch(g: Optional[Gaussians], batch: Batch, opts: Opts, headroom: float = 1.25,
                    min_capacity: int = 1024, stream=None) -> Bins:
    """Workspace for the batch with room for its exact key count times ``headroom`` (g None: the
    batch's own sets)."""
    probe = Bins(0, batch, opts, 0, device="cuda")
    k = gs_bin_query_batch(g, batch, opts, probe, stream)
    return Bins(0, batch, opts, max(min_capacity, int(math.ceil(k * headroom))), device=probe.ws.device)


def concat(gs_: Sequence[Gaussians]) -> Gaussians:
    """One Gaussian set holding the given sets in order (the batch layout)."""
    cat = lambda k: torch.cat([getattr(x, k).contiguous() for x in gs_])  # noqa: E731
    relax = None
    if any(x.relax is not None for x in gs_):
        relax = torch.cat([x.relax if x.relax is not None else torch.ones_like(x.amp) for x in gs_]).contiguous()
    return Gaussians(cat("mu"), cat("log_scale"), cat("quat"), cat("amp"), relax)


def render_batch(g: Optional[Gaussians], batch: Batch, opts: Optional[Opts] = None, bins: Optional[Bins] = None,
                 want_w: bool = True, stream=None):
    """Bin + forward of every scan of the batch in one launch per phase.  Returns the concatenated
    (I, W) (flat float32) and the bins; ``batch.split`` gives the per-scan volumes."""
    opts = opts or Opts()
    if bins is None:
        bins = plan_bins_batch(g, batch, opts, stream=stream)
    dev = bins.ws.device
    nv = batch.v_offsets[-1]
    I = torch.empty(nv, dtype=torch.float32, device=dev)
    W = torch.empty(nv, dtype=torch.float32, device=dev) if want_w else None
    gs_bin_batch(g, batch, opts, bins, stream)
    gs_render_fwd_batch(g, batch, opts, bins, I, W, stream)
    return I, W, bins


def render(g: Gaussians, grid: Grid, opts: Optional[Opts] = None, bins: Optional[Bins] = None, want_w: bool = True,
           stream=None):
    """Bin + forward.  Returns (I, W, bins) with I, W float32 [nz, ny, nx] (W None if not wanted)."""
    opts = opts or Opts()
    if bins is None:
        bins = plan_bins(g, grid, opts, stream=stream)
    dev = bins.ws.device
    I = torch.empty(grid.shape, dtype=torch.float32, device=dev)
    W = torch.empty(grid.shape, dtype=torch.float32, device=dev) if want_w else None
    gs_bin(g, grid, opts, bins, stream)
    gs_render_fwd(g, grid, opts, bins, I, W, stream)
    return I, W, bins


def backward(g: Gaussians, grid: Grid, opts: Opts, bins: Bins, I, W, dL_dI, stream=None) -> Grads:
    grads = Grads.empty(g.n, relax=g.relax is not None, device=bins.ws.device)
    gs_render_bwd(g, grid, opts, bins, I, W, dL_dI, grads, stream)
    return grads


@dataclass
class Adam:
    lr: Sequence[float] = (1e-2, 5e-3, 1e-3, 1e-2, 0.0)
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self) -> gs_adam_t:
        return gs_adam_t((ctypes.c_float * 5)(*self.lr), self.beta1, self.beta2, self.eps)


class FitState:
    """Parameters (updated in place), Adam moments and the device step counter(s) of a fit (one
    counter per scan of a batch)."""

    def __init__(self, g: Gaussians, nscans: int = 1):
        self.g = g
        n = g.n
        dev = g.amp.device
        self.m = torch.zeros(12 * n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(12 * n, dtype=torch.float32, device=dev)
        self.step = torch.zeros(nscans, dtype=torch.int32, device=dev)

    def c(self) -> gs_fit_state_t:
        g = self.g
        return gs_fit_state_t(g.n, _ptr(g.mu), _ptr(g.log_scale), _ptr(g.quat), _ptr(g.amp), _ptr(g.relax),
                              _ptr(self.m), _ptr(self.v), _ptr(self.step))


def gs_adam_step(st: FitState, grads: Grads, hp: Adam, bins: Optional[Bins] = None, stream=None) -> None:
    _check(_lib.gs_adam_step(ctypes.byref(st.c()), ctypes.byref(grads.c()), ctypes.byref(hp.c()),
                             ctypes.byref(bins.c()) if bins is not None else None, _stream(stream)))


class FitBuffers:
    """Per-step buffers of a fit on one grid, or on a batch (``grid`` a Batch: concatenated flat
    volumes, one loss per scan)."""

    def __init__(self, n: int, grid, relax: bool, device="cuda", need_dL_dI: bool = True):
        f = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)  # noqa: E731
        if isinstance(grid, Batch):
            shape, nloss, n = (grid.v_offsets[-1],), len(grid), grid.n_total
            sb = gs_fit_scratch_bytes_batch(grid)
        else:
            shape, nloss = grid.shape, 1
            sb = max(gs_loss_scratch_bytes(grid.size), gs_fit_scratch_bytes(grid))
        self.I, self.W = f(shape), f(shape)
        self.dL_dI = f(shape) if need_dL_dI else None
        self.grads = Grads.empty(n, relax, device)
        self.scratch = torch.empty(sb, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(nloss, dtype=torch.float32, device=device)

    def c(self) -> gs_fit_buffers_t:
        return gs_fit_buffers_t(_ptr(self.I), _ptr(self.W), _ptr(self.dL_dI), self.grads.c(), _ptr(self.scratch),
                                self.scratch.numel(), _ptr(self.loss))


@dataclass
class FitOpts:
    """Fit options; ``grid`` is the HR grid of a single-scan fit (a batch carries its own grids and
    may leave it None)."""

    grid: Optional[Grid] = None
    opts: Opts = field(default_factory=Opts)
    zdown: int = 4
    adam: Adam = field(default_factory=Adam)

    def c(self) -> gs_fit_opts_t:
        grid = self.grid if self.grid is not None else Grid(1, 1, 1)
        return gs_fit_opts_t(grid.c(), self.opts.c(), self.zdown, 0, self.adam.c())


def gs_fit_step(st: FitState, lr_obs: torch.Tensor, fo: FitOpts, bins: Bins, buf: FitBuffers, stream=None) -> None:
    _check(_lib.gs_fit_step(ctypes.byref(st.c()), _ptr(_f32(lr_obs)), ctypes.byref(fo.c()), ctypes.byref(bins.c()),
                            ctypes.byref(buf.c()), _stream(stream)))


def gs_fit_step_batch(st: FitState, lr_obs: torch.Tensor, batch: Batch, fo: FitOpts, bins: Bins, buf: FitBuffers,
                      stream=None) -> None:
    _check(_lib.gs_fit_step_batch(ctypes.byref(st.c()), _ptr(_f32(lr_obs)), ctypes.byref(batch.c()),
                                  ctypes.byref(fo.c()), ctypes.byref(bins.c()), ctypes.byref(buf.c()),
                                  _stream(stream)))
