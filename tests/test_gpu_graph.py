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
    assert entry["bx"] == opts.bx and set(entry["ms"]) == {str(b) for b in autotune.CANDIDATES}
    # a second tuner reads the cache and measures nothing
    t2 = autotune.Tuner(path)
    t2._time = None  # would raise if called
    assert t2.fit_opts(g, batch, obs, zdown=4).bx == opts.bx
    ropts = t.render_opts(g, batch, steps=2)
    assert ropts.bx in autotune.CANDIDATES
