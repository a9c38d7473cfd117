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
    for bad in (gs.Opts(cutoff=0.0), gs.Opts(eps=-1.0), gs.Opts(cutoff=float("inf"))):
        with pytest.raises(gs.GSError) as e:
            gs.gs_workspace_size(10, g, bad, 10)
        assert e.value.code == gs.GS_ERR_INVALID_ARG
    with pytest.raises(gs.GSError) as e:
        gs.gs_workspace_size(10, g, gs.Opts(bx=5), 10)
    assert e.value.code == gs.GS_ERR_UNSUPPORTED
    assert "not supported" in gs.gs_last_error()


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
