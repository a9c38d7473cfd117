"""The continuous-batching request loop: every result equals the same request run alone, also
under an HBM budget low enough to force queueing."""
import numpy as np
import pytest
import torch

from paper_2603_09621_amd import synth
from tests.gpu_util import gs_mod, say

pytestmark = pytest.mark.gpu

SCALES = (1.5, 2.0, 2.5)


def _world(seed=41):
    gs = gs_mod()
    sets, dims = [], []
    for k, (n, box) in enumerate(((3000, (16, 16, 12)), (6000, (20, 18, 10)), (1500, (12, 14, 16)))):
        ell = (np.prod(box) / n) ** (1 / 3)
        p = synth.gaussians_uniform((seed, k), n, box, ls_mean=float(np.log(0.75 * ell)), ls_std=0.3)
        sets.append(gs.Gaussians.from_numpy(p))
        dims.append(box)
    fits = []
    for k, (d, n) in enumerate((((32, 24, 16), 500), ((24, 32, 8), 300))):
        lr = synth.zmean_observation(synth.phantom((seed, 9, k), d), 4)
        fits.append((synth.lattice_init((seed, 10, k), lr, n, 4), lr, d))
    return sets, dims, fits


def _requests(fits, nrender=12, seed=42, spacing=0.002, steps=(7, 4)):
    from paper_2603_09621_amd import serve

    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(nrender):
        reqs.append(serve.RenderRequest(int(rng.integers(3)), float(SCALES[int(rng.integers(len(SCALES)))]),
                                        arrival=i * spacing))
    for k, (p, lr, d) in enumerate(fits):  # fits arrive at different times and run different lengths
        reqs.append(serve.FitRequest(p, lr, d, steps=steps[k], arrival=(2 + 5 * k) * spacing))
    return reqs


def _alone_render(gs, g, grid):
    I, _, bins = gs.render(g, grid, gs.Opts(), want_w=False)
    gs.gs_status(bins)
    return I.reshape(-1)


def _alone_fit(gs, p, lr, d, steps):
    g = gs.Gaussians.from_numpy(p)
    grid = gs.Grid(*d)
    fo = gs.FitOpts(grid)
    bins = gs.plan_bins(g, grid, fo.opts, headroom=1.5)
    st = gs.FitState(g)
    buf = gs.FitBuffers(g.n, grid, relax=True)
    obs = torch.from_numpy(lr).cuda()
    for _ in range(steps):
        gs.gs_fit_step(st, obs, fo, bins, buf)
    gs.gs_status(bins)
    return g, float(buf.loss.item())


def _check(gs, server, reqs, sets, results=None):
    """Every result (on the device, or copied to the host by the loop's on_done) bitwise equal to the
    same request run alone."""
    assert len(server.done) == len(reqs)
    for r in reqs:
        res = r.result if results is None else results[r.rid]
        if r.kind == "render":
            want = _alone_render(gs, sets[r.set_id], r.grid)
            assert torch.equal(res.reshape(-1), want.to(res.device)), f"render {r.rid} differs from the same render alone"
        else:
            g, loss = _alone_fit(gs, r.params, r.lr_obs, r.dims, r.steps)
            for k in gs.GROUPS:
                assert torch.equal(res[k], getattr(g, k).to(res[k].device)), f"fit {r.rid}: {k} differs from the fit alone"
            assert r.loss == loss


def test_results_equal_alone_and_in_the_mix():
    gs = gs_mod()
    from paper_2603_09621_amd import serve

    sets, dims, fits = _world()
    server = serve.Server(sets, dims, hbm_budget=8 << 30, fit_chunk=3)
    reqs = _requests(fits)
    say("serve mix", len(reqs))
    rep = server.run(reqs, realtime=True)
    say(rep)
    assert rep["render"]["count"] == 12 and rep["fit"]["count"] == 2
    assert rep["render"]["p99_ms"] >= rep["render"]["p50_ms"] > 0
    _check(gs, server, reqs, sets)


def test_low_hbm_budget_forces_queueing():
    gs = gs_mod()
    from paper_2603_09621_amd import serve

    sets, dims, fits = _world(43)
    probe = serve.Server(sets, dims, hbm_budget=1 << 40)
    reqs = _requests(fits, seed=44, spacing=0.0)
    fps = []
    for r in reqs:
        if r.kind == "render":
            r.grid = probe.render_grid(r.set_id, r.scale)
            fps.append(probe.render_footprint(r))
        else:
            probe.prepare_fit(r)
            fps.append(r.footprint)
    budget = max(fps) + min(fps) // 2  # the largest request plus a little: requests must queue
    server = serve.Server(sets, dims, hbm_budget=budget, fit_chunk=2, keep_results=False)
    say("serve low budget", budget, len(reqs))
    results = {}

    def to_host(r):  # results leave the device as they complete, so device memory is the loop's own
        results[r.rid] = r.result.cpu() if r.kind == "render" else {k: v.cpu() for k, v in r.result.items()}

    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    rep = server.run(reqs, realtime=False, on_done=to_host)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    say(rep, "device peak above the resident sets", peak)
    assert server.peak_used <= budget
    assert peak <= budget, f"the loop held {peak} bytes of device memory at once, over its budget {budget}"
    waited = sum(1 for r in reqs if r.t_admit > 0.0005)
    assert waited >= len(reqs) // 2, "a low budget should hold most requests in the queue"
    _check(gs, server, reqs, sets, results)
