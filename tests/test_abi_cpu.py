"""C-ABI checks that need no GPU: the library loads, exports every entry point include/gs.h
declares, and its host-side argument checks and workspace sizing behave."""
import ctypes
import os
import re

import pytest

from paper_2603_09621_amd import gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(gs.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(gs.EXPORTED)


def test_invalid_arguments_are_rejected():
    g = gs.Grid(16, 16, 8)
    with pytest.raises(gs.GSError) as e:
        gs.gs_workspace_size(-1, g, gs.Opts(), 10)
    assert e.value.code == gs.GS_ERR_INVALID_ARG
    for bad in (gs.Grid(0, 4, 4), gs.Grid(4, 4, 4, spacing=(1, 0, 1)), gs.Grid(4, 4, 4, spacing=(1, float("nan"), 1))):
        with pytest.raises(gs.GSError) as e:
            gs.gs_workspace_size(10, bad, gs.Opts(), 10)
        assert e.value.code == gs.GS_ERR_INVALID_ARG
    for bad in (gs.Opts(cutoff=0.0), gs.Opts(eps=-1.0), gs.Opts(eps=0.0), gs.Opts(cutoff=float("inf"))):
        with pytest.raises(gs.GSError) as e:
            gs.gs_workspace_size(10, g, bad, 10)
        assert e.value.code == gs.GS_ERR_INVALID_ARG
    with pytest.raises(gs.GSError) as e:
        gs.gs_workspace_size(10, g, gs.Opts(bx=5), 10)
    assert e.value.code == gs.GS_ERR_UNSUPPORTED
    assert "not supported" in gs.gs_last_error()
    # voxel boxes are kept in 16-bit indices: at most 65535 voxels per axis
    assert gs.gs_workspace_size(10, gs.Grid(65535, 4, 4), gs.Opts(), 10) > 0
    with pytest.raises(gs.GSError) as e:
        gs.gs_workspace_size(10, gs.Grid(4, 65536, 4), gs.Opts(), 10)
    assert e.value.code == gs.GS_ERR_UNSUPPORTED


def test_workspace_grows_with_n_and_capacity():
    g = gs.Grid(64, 64, 32)
    o = gs.Opts()
    a = gs.gs_workspace_size(1000, g, o, 0)
    b = gs.gs_workspace_size(2000, g, o, 0)
    c = gs.gs_workspace_size(2000, g, o, 100000)
    assert 0 < a < b < c
    # per key: the two uint32 brick lists + 48 B of partial sums
    assert c - b >= 100000 * (2 * 4 + 48)
    assert gs.gs_loss_scratch_bytes(1) >= 4
    assert gs.gs_loss_scratch_bytes(10 ** 7) >= 4 * (10 ** 7 // 4096)


def test_brick_shapes():
    for bx in (4, 8, 16):
        assert gs.brick_supported(bx, 8, 4)
    for shape in ((8, 4, 4), (8, 8, 8), (2, 8, 4), (32, 8, 4), (12, 8, 4)):
        assert not gs.brick_supported(*shape)


def test_batch_sizes_and_checks():
    o = gs.Opts()
    grids = [gs.Grid(24, 16, 8), gs.Grid(40, 8, 12), gs.Grid(8, 8, 4)]
    ns = [100, 0, 37]
    b = gs.Batch(ns, grids)
    # a batch of one scan sizes like the single-scan call
    for k in range(3):
        one = gs.Batch([ns[k]], [grids[k]])
        assert gs.gs_workspace_size_batch(one, o, 500) == gs.gs_workspace_size(ns[k], grids[k], o, 500)
        assert gs.gs_fit_scratch_bytes_batch(one) == gs.gs_fit_scratch_bytes(grids[k])
    whole = gs.gs_workspace_size_batch(b, o, 500)
    assert whole >= gs.gs_workspace_size(sum(ns), grids[0], o, 500)
    # fit scratch: one float per brick of the narrowest brick shape, summed over the scans
    bricks4 = sum(-(-g.nx // 4) * -(-g.ny // 8) * -(-g.nz // 4) for g in grids)
    assert gs.gs_fit_scratch_bytes_batch(b) >= 4 * bricks4
    for bad in (gs.Batch([], []), gs.Batch([1] * 17, [grids[0]] * 17), gs.Batch([-1], [grids[0]]),
                gs.Batch([1], [gs.Grid(0, 4, 4)])):
        with pytest.raises(gs.GSError) as e:
            gs.gs_workspace_size_batch(bad, o, 10)
        assert e.value.code == gs.GS_ERR_INVALID_ARG
    assert gs.gs_fit_scratch_bytes_batch(gs.Batch([], [])) == 0


def test_forward_only_workspace():
    g = gs.Grid(64, 64, 32)
    full = gs.gs_workspace_size(5000, g, gs.Opts(), 200000)
    fwd = gs.gs_workspace_size(5000, g, gs.Opts(forward_only=True), 200000)
    assert full - fwd >= 200000 * 48
    bad = gs.gs_opts_t(8, 8, 4, 3.0, 1e-8, 2)  # unknown flag bit
    out = ctypes.c_size_t(0)
    rc = gs._lib.gs_workspace_size(10, ctypes.byref(g.c()), ctypes.byref(bad), 10, ctypes.byref(out))
    assert rc == gs.GS_ERR_INVALID_ARG and "flags" in gs.gs_last_error()


def test_binding_exposes_the_conveniences():
    """The binding's public classes and helpers are all there (no GPU needed to look them up)."""
    for name in ("Grid", "Opts", "Gaussians", "Batch", "Bins", "Grads", "Adam", "FitState", "FitBuffers",
                 "FitOpts", "render", "render_batch", "backward", "plan_bins", "plan_bins_batch", "concat",
                 "gs_fit_step", "gs_fit_step_batch", "gs_render_bwd_batch", "gs_count_pairs_batch"):
        assert hasattr(gs, name), name
    from paper_2603_09621_amd import autograd, autotune, graph, serve  # noqa: F401  (import cleanly)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """Importing the binding where libgs.so is absent raises ImportError (there is no fallback)."""
    import shutil
    import subprocess
    import sys

    pkg = tmp_path / "pkg_copy"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2603_09621_amd", "gs.py"), pkg / "gs.py")
    code = "import sys; sys.path.insert(0, %r); import gs" % str(pkg)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libgs.so is missing" in r.stderr


def test_noalloc_rejects_sets_beyond_the_static_scratch():
    """The no-allocation render refuses, before touching any device, a set whose per-Gaussian
    workspace alone exceeds the static scratch (the pointers are never dereferenced)."""
    fake = ctypes.c_void_p(256)
    n = 2_000_000  # 2M x (48 + 32 + 4 + 32 + 16) B of records, offsets, run cache and boxes > 64 MiB
    g = gs.gs_gaussians_t(n, fake, fake, fake, fake, None)
    grid = gs.Grid(64, 64, 32).c()
    opts = gs.Opts().c()
    rc = gs._lib.gs_render_fwd_noalloc(ctypes.byref(g), ctypes.byref(grid), ctypes.byref(opts), fake, None, None, None)
    assert rc == gs.GS_ERR_INVALID_ARG
    assert "static scratch" in gs.gs_last_error()
    m = re.search(r"#define GS_STATIC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", open(os.path.join(ROOT, "include", "gs.h")).read())
    assert m and gs.GS_STATIC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
    rc = gs._lib.gs_render_fwd_noalloc(ctypes.byref(g), ctypes.byref(grid), ctypes.byref(opts), None, None, None, None)
    assert rc == gs.GS_ERR_INVALID_ARG


def test_tuning_flags_are_checked():
    """The tuning bits are accepted (one emit stage and one backward group size at most); other bits
    are rejected."""
    g = gs.Grid(16, 16, 8)
    for o in (gs.Opts(bwd_bricks=1), gs.Opts(bwd_bricks=2), gs.Opts(bwd_window=256), gs.Opts(emit_stage=4096),
              gs.Opts(emit_stage=6144), gs.Opts(bwd_bricks=1, bwd_window=256, emit_stage=6144, forward_only=True)):
        assert gs.gs_workspace_size(10, g, o, 10) > 0
    out = ctypes.c_size_t(0)
    for both in (gs.FLAG_EMIT_STAGE_4K | gs.FLAG_EMIT_STAGE_6K, gs.FLAG_BWD_ONE_BRICK | gs.FLAG_BWD_TWO_BRICKS):
        bad = gs.gs_opts_t(8, 8, 4, 3.0, 1e-8, both)
        assert gs._lib.gs_workspace_size(10, ctypes.byref(g.c()), ctypes.byref(bad), 10, ctypes.byref(out)) == \
            gs.GS_ERR_INVALID_ARG
    for bit in (1 << 1, 1 << 9, 1 << 31):
        bad = gs.gs_opts_t(8, 8, 4, 3.0, 1e-8, bit)
        assert gs._lib.gs_workspace_size(10, ctypes.byref(g.c()), ctypes.byref(bad), 10, ctypes.byref(out)) == \
            gs.GS_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        gs.Opts(bwd_bricks=3).c()
