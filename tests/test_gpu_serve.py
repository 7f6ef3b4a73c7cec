"""Serving form: continuous batching with admission by HBM footprint.

Each request's effective toughness is the same alone (a handle of its own)
and in the mix (a slot of a shared batched pool, admitted while other
requests run, pools stepping concurrently on their own streams).
"""
import numpy as np
import pytest

from paper_2508_07424_amd import workloads as W

pytestmark = pytest.mark.gpu


def _requests(count=6, seed=11):
    from paper_2508_07424_amd.serve import Request
    stream = W.serving_stream(count, seed=seed, sizes_2d=(32, 48), sizes_3d=(16,), frac_3d=0.2,
                              rate=50.0, dtau_frac=0.02)
    return [Request(i, w, arrival=a, max_steps=300) for i, (a, w) in enumerate(stream)]


def test_alone_equals_in_the_mix_fp64():
    from paper_2508_07424_amd import mirve
    from paper_2508_07424_amd.serve import Server, serve_sequential
    reqs = _requests()
    alone = serve_sequential(reqs, precision=mirve.RVE_PREC_FP64)
    srv = Server(precision=mirve.RVE_PREC_FP64, slots_per_pool=2)
    try:
        mixed = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    print("pools opened, stalls", srv.stalls, "ticks", srv.ticks, flush=True)
    for a, m in zip(alone, mixed):
        print(a.rid, reqs[a.rid].workload.n, a.steps, m.steps, a.G_eff, m.G_eff, flush=True)
        assert a.status == 0 and m.status == 0
        assert a.steps == m.steps
        assert abs(a.G_eff - m.G_eff) <= 1e-9 * abs(a.G_eff)


def test_alone_equals_in_the_mix_mixed_precision():
    """The same in the precision form: each request's G_eff served as a slot
    of a shared mixed-precision pool equals its G_eff alone in a mixed
    handle of its own within the toughness bar of 1e-3 (the launch shape of
    a pool may differ from a single slot's, which changes the summation
    order of the partial sums)."""
    from paper_2508_07424_amd import mirve
    from paper_2508_07424_amd.serve import Server, serve_sequential
    reqs = _requests()
    alone = serve_sequential(reqs, precision=mirve.RVE_PREC_MIXED)
    srv = Server(precision=mirve.RVE_PREC_MIXED, slots_per_pool=2)
    try:
        mixed = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    for a, m in zip(alone, mixed):
        print(a.rid, reqs[a.rid].workload.n, a.steps, m.steps, a.G_eff, m.G_eff, flush=True)
        assert a.status == 0 and m.status == 0
        assert abs(a.G_eff - m.G_eff) <= 1e-3 * abs(a.G_eff)


def test_admission_respects_the_budget():
    from paper_2508_07424_amd import mirve
    from paper_2508_07424_amd.serve import Server
    reqs = _requests(count=5, seed=4)
    srv = Server(precision=mirve.RVE_PREC_MIXED, slots_per_pool=2, budget_bytes=1)
    # room for about one two-slot pool at a time: requests of other classes wait
    budget = int(1.05 * max(srv.footprint(r.workload, 2) for r in reqs))
    assert len({tuple(r.workload.n) for r in reqs}) > 1
    srv.budget = budget
    try:
        res = srv.run(reqs, realtime=False)
    finally:
        srv.close()
    print("stalls", srv.stalls, "peak", srv.peak_bytes, "budget", budget, flush=True)
    for r in res:
        print(r, reqs[r.rid].workload.n, flush=True)
    assert srv.peak_bytes <= budget
    # every request ran to its end (the fracture point, or the step limit)
    assert all(r.status in (0, mirve.RVE_ENOTDONE) for r in res)
    assert sum(r.G_eff is not None for r in res) >= len(res) - 1
    assert srv.stalls > 0
