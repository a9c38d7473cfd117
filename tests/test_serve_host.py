"""Host-side rules of the request loop (no GPU): admission by slots and HBM budget, and the moment
layout used when fits are packed into one batch."""
import numpy as np

from paper_2603_09621_amd import serve


class _Req:
    def __init__(self, kind, footprint):
        self.kind, self.footprint = kind, footprint


def _server(budget, **kw):
    return serve.Server([], [], hbm_budget=budget, device="cpu", **kw)


def test_admission_respects_budget_and_slots():
    s = _server(1000, max_batch=2, max_fits=1)
    r = _Req("render", 600)
    assert s.admissible(r, busy=False, renders_waiting=0, fits_active=0)
    s.used = 600
    assert not s.admissible(_Req("render", 500), busy=True, renders_waiting=1, fits_active=0)
    assert s.admissible(_Req("render", 400), busy=True, renders_waiting=1, fits_active=0)
    # a request larger than the whole budget runs alone
    s.used = 0
    assert s.admissible(_Req("fit", 5000), busy=False, renders_waiting=0, fits_active=0)
    assert not s.admissible(_Req("fit", 5000), busy=True, renders_waiting=0, fits_active=0)
    # slots
    assert not s.admissible(_Req("fit", 1), busy=True, renders_waiting=0, fits_active=1)
    assert not s.admissible(_Req("render", 1), busy=True, renders_waiting=8, fits_active=0)


def test_group_slices_cover_the_moment_layout():
    """mu 3n, log_scale 3n, quat 4n, amp n, relax n: contiguous and exhaustive over 12 n."""
    n = 7
    covered = np.zeros(12 * n, dtype=int)
    for off, w in serve.GROUP_SLICES:
        covered[off * n:(off + w) * n] += 1
    assert (covered == 1).all()
