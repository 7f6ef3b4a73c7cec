"""The allocation-free Green operator (rve_apply_green_op_device_noalloc)
against the workspace form (rve_apply_green_op_device) through the C ABI.

Both run the same kernels on the same handle; only the buffers that hold
the spectrum and the per-block partial sums differ (the library's static
device array against the handle's workspace), so the outputs must agree
bit for bit.  Two calls in a row, the second on a smaller handle (the
array keeps the first call's contents), then a handle too large for the
array is refused before any work.
"""
import numpy as np
import pytest

from paper_2508_07424_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compare(m, wls, prec, repeat):
    import torch
    stream = torch.cuda.Stream()
    r = m.from_workloads(wls, precision=prec, stream=stream)
    # a non-trivial damage field: one dissipation step of every slot
    infos, st = r.rve_run_slots([w.dtau for w in wls], [1] * len(wls))
    assert all(s == 0 for s in st), st
    dt = torch.float64 if prec == m.RVE_PREC_FP64 else torch.float32
    n = r.B * r.s * r.N
    with torch.cuda.stream(stream):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(17)
        eps = torch.randn(n, dtype=dt, device="cuda", generator=gen)
        ref = torch.full_like(eps, float("nan"))
        out = torch.full_like(eps, float("nan"))
    stream.synchronize()
    print("handle", wls[0].n, "batch", r.B, "precision", prec, "repeat", repeat, flush=True)
    r.rve_apply_green_op_device(eps, ref, repeat)
    r.rve_apply_green_op_device_noalloc(eps, out, repeat)
    stream.synchronize()
    a, b = ref.cpu().numpy(), out.cpu().numpy()
    assert np.all(np.isfinite(a))
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    # the same field through the host form of the operator (slot 0)
    host = r.rve_apply_green_op(eps[: r.s * r.N].double().cpu().numpy().reshape((r.s,) + r.shape))
    if repeat == 1:
        den = np.max(np.abs(host))
        tol = 1e-12 if prec == m.RVE_PREC_FP64 else 1e-5
        assert np.max(np.abs(b[: r.s * r.N].reshape(host.shape) - host)) <= tol * den
    r.close()


def test_noalloc_matches_workspace_form_two_calls():
    from paper_2508_07424_amd import mirve as m
    big = [W.composite_2d(n=128, seed=s, E_ratio=5.0, Gc_ratio=2.0, vf=0.3, ell=2.0, crack=20)
           for s in (1, 2, 3)]
    _compare(m, big, m.RVE_PREC_FP64, 1)
    small = [W.homogeneous_2d(nx=48, ny=40, crack=8)]
    _compare(m, small, m.RVE_PREC_MIXED, 3)


def test_noalloc_refuses_a_handle_beyond_the_array():
    import torch
    from paper_2508_07424_amd import mirve as m
    # 3 x 129 x 256 x 16 B = 1.59 MB of FP64 spectrum per 256^2 slot: 48 slots
    # exceed the 64 MiB array
    cfg = m.make_config((256, 256), batch=48)
    r = m.Rve(cfg, stream=torch.cuda.Stream())
    eps = torch.zeros(r.B * r.s * r.N, dtype=torch.float64, device="cuda")
    out = torch.empty_like(eps)
    with pytest.raises(m.MirveError) as e:
        r.rve_apply_green_op_device_noalloc(eps, out, 1)
    assert e.value.code == m.RVE_ENOSPC
    print(m.lib.rve_last_error(r.h).decode(), flush=True)
    r.close()
