"""HIP-graph replay of batched fit steps and the brick-width autotuner."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2603_09621_amd import synth
from tests.gpu_util import gs_mod, say

pytestmark = pytest.mark.gpu

SCANS = [(231, (32, 24, 16), 500), (232, (24, 40, 8), 300), (233, (40, 16, 12), 400)]


def _batch(zdown=4):
    gs = gs_mod()
    data = []
    for seed, dims, n in SCANS:
        hr = synth.phantom(seed, dims)
        lr = synth.zmean_observation(hr, zdown)
        data.append((synth.lattice_init(seed + 1, lr, n, f=zdown), lr, dims))
    batch = gs.Batch([p["amp"].shape[0] for p, _, _ in data], [gs.Grid(*d) for _, _, d in data])
    obs = torch.from_numpy(np.concatenate([lr.reshape(-1) for _, lr, _ in data])).cuda()
    return data, batch, obs


def _state(data, batch, opts, zdown):
    gs = gs_mod()
    g = gs.concat([gs.Gaussians.from_numpy(p) for p, _, _ in data])
    fo = gs.FitOpts(None, opts=opts, zdown=zdown)
    bins = gs.plan_bins_batch(g, batch, opts, headroom=2.0)
    st = gs.FitState(g, nscans=len(batch))
    buf = gs.FitBuffers(g.n, batch, relax=True, need_dL_dI=zdown != opts.bz)
    return g, fo, bins, st, buf


@pytest.mark.parametrize("zdown", (4, 2))
def test_graph_replays_equal_eager_steps(zdown):
    gs = gs_mod()
    from paper_2603_09621_amd import graph

    data, batch, obs = _batch(zdown)
    say("graph replay", zdown, batch.ns)
    A = _state(data, batch, gs.Opts(), zdown)
    B = _state(data, batch, gs.Opts(), zdown)
    for g, fo, bins, st, buf in (A, B):  # eager first step: kernels loaded before capture
        gs.gs_fit_step_batch(st, obs, batch, fo, bins, buf)
    fg = graph.FitGraph(A[3], obs, batch, A[1], A[2], A[4], steps=2)
    for r in range(3):
        fg.replay()
        for _ in range(2):
            gs.gs_fit_step_batch(B[3], obs, batch, B[1], B[2], B[4])
        # unrelated eager work and a synchronisation between replays
        x = torch.randn(256, 256, device="cuda")
        (x @ x).sum().item()
        torch.cuda.synchronize()
        gs.gs_status(A[2])
        for k in gs.GROUPS:
            assert torch.equal(getattr(A[0], k), getattr(B[0], k)), f"replay {r}: {k}"
        assert torch.equal(A[3].m, B[3].m) and torch.equal(A[3].v, B[3].v), f"replay {r}: moments"
        assert torch.equal(A[3].step, B[3].step), f"replay {r}: steps"
        assert torch.equal(A[4].loss, B[4].loss), f"replay {r}: loss"
        assert int(A[3].step[0].item()) == 1 + 2 * (r + 1)


def test_autotuner_picks_and_caches(tmp_path):
    gs = gs_mod()
    from paper_2603_09621_amd import autotune

    data, batch, obs = _batch(4)
    g = gs.concat([gs.Gaussians.from_numpy(p) for p, _, _ in data])
    before = {k: getattr(g, k).clone() for k in gs.GROUPS}
    path = os.path.join(tmp_path, "tune.json")
    t = autotune.Tuner(path)
    say("autotune", batch.ns)
    opts = t.fit_opts(g, batch, obs, zdown=4, steps=2)
    assert opts.bx in autotune.CANDIDATES
    for k in gs.GROUPS:  # the tuner works on copies
        assert torch.equal(getattr(g, k), before[k])
    rec = json.load(open(path))
    assert len(rec) == 1
    (entry,) = rec.values()
    assert entry["opts"] == opts.tuning
    # every width was timed, and every value of each result-invariant knob at the chosen width
    widths = {k.split("/")[0] for k in entry["ms"]}
    assert widths == {f"bx{b}" for b in autotune.CANDIDATES}
    assert {k for k in entry["ms"] if k.startswith(f"bx{opts.bx}/")} >= {
        f"bx{opts.bx}/g{g_}/w512/e0" for g_ in (8, 2, 1)}
    assert opts.bwd_bricks in (8, 2, 1) and opts.bwd_window in (256, 512) and opts.emit_stage in (0, 4096, 6144)
    # a second tuner reads the cache and measures nothing
    t2 = autotune.Tuner(path)
    t2._time = None  # would raise if called
    assert t2.fit_opts(g, batch, obs, zdown=4).tuning == opts.tuning
    ropts = t.render_opts(g, batch, steps=2)
    assert ropts.bx in autotune.CANDIDATES


def test_tuning_knobs_leave_results_bitwise_equal():
    """Bricks per backward workgroup, the backward's ordering window and the emit's stage change speed
    only: renders, gradients and fit steps are bitwise those of the defaults, at every width."""
    gs = gs_mod()
    data, batch, obs = _batch(4)
    variants = [dict(), dict(bwd_bricks=2), dict(bwd_bricks=1), dict(bwd_window=256), dict(bwd_bricks=2, bwd_window=256),
                dict(bwd_bricks=1, bwd_window=256), dict(emit_stage=4096), dict(emit_stage=6144)]
    for bx in (4, 8, 16):
        ref = None
        for kw in variants:
            opts = gs.Opts(bx=bx, **kw)
            g = gs.concat([gs.Gaussians.from_numpy(p) for p, _, _ in data])
            bins = gs.plan_bins_batch(g, batch, opts, headroom=1.5)
            st = gs.FitState(g, nscans=len(batch))
            buf = gs.FitBuffers(g.n, batch, relax=g.relax is not None, device="cuda", need_dL_dI=False)
            fo = gs.FitOpts(None, opts=opts, zdown=4)
            for _ in range(2):
                gs.gs_fit_step_batch(st, obs, batch, fo, bins, buf)
            gs.gs_status(bins)
            ev = torch.zeros(6, dtype=torch.int64, device="cuda")
            gs.gs_count_pairs_batch(g, batch, opts, bins, ev[:1])
            out = {k: getattr(g, k).clone() for k in gs.GROUPS if getattr(g, k) is not None}
            out.update(I=buf.I.clone(), W=buf.W.clone(), loss=buf.loss.clone(), pairs=ev[:1].clone(),
                       **{f"d_{k}": v.clone() for k, v in buf.grads.as_dict().items() if v is not None})
            if ref is None:
                ref = out
                continue
            for k in ref:
                assert torch.equal(out[k], ref[k]), f"bx {bx} {kw}: {k} differs from the default options"
