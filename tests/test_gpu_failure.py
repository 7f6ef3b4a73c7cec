"""Failure handling and checkpoints of the C ABI on the GPU.

- A step whose solve cannot converge returns RVE_ENOCONV with the reason of
  the failure, and the committed state (phi, history, E, Sigma, T, tau,
  step) is bitwise what it was before the call, also when sub-steps of a
  halved step had committed before the failure (Sec. 4.1: dissipation
  control allows any subdivision of the increment; the step as a whole is
  transactional).
- Non-finite inputs are rejected with RVE_EINVAL before any work.
- A saved state, loaded into a fresh handle with the same microstructure,
  continues bit for bit as the original handle does.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2508_07424_amd import workloads as W

pytestmark = pytest.mark.gpu


def _snapshot(r, slot=0):
    return (r.rve_get_field("phi", slot=slot), r.rve_get_field("hist", slot=slot),
            r.rve_get_scalars(slot=slot))


def _same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    for key in ("E", "Sigma", "T", "tau", "tau0", "step", "fractured"):
        assert a[2][key] == b[2][key], key


def test_cg_limit_leaves_state_unchanged():
    from paper_2508_07424_amd import mirve as m
    w = W.composite_2d_small()
    r = m.from_workload(w, max_cg=1, max_halvings=2)
    before = _snapshot(r)
    info, st = r.rve_run_slots([w.dtau], [1])
    print("status", st, "reason", m.WHY[info[0]["reason"]], m.lib.rve_last_error(r.h), flush=True)
    assert st[0] == m.RVE_ENOCONV and info[0]["reason"] == 2     # RVE_WHY_CG
    assert info[0]["n_steps"] == 0
    _same(before, _snapshot(r))


def test_stagger_limit_leaves_state_unchanged():
    from paper_2508_07424_amd import mirve as m
    w = W.composite_2d_small()
    r = m.from_workload(w, max_stagger=1, max_halvings=0)
    before = _snapshot(r)
    with pytest.raises(m.MirveError) as e:
        r.rve_step_dissipation(w.dtau)
    assert e.value.code == m.RVE_ENOCONV
    _same(before, _snapshot(r))


def test_failure_after_committed_substeps_rolls_back():
    """Steps near the unstable crack advance of the 64 x 64 composite, with
    increments up to 4 dtau and a single halving level: the full increment
    fails, its first half commits and the second half fails for good.  Every
    failed call must leave the state exactly as it was before the call, and
    the scan must meet at least one such roll-back."""
    from paper_2508_07424_amd import mirve as m
    w = W.composite_2d_small()
    base = m.from_workload(w)
    blobs = {}
    for k in range(1, 67):
        base.rve_step_dissipation(w.dtau)
        if k in (56, 62, 66):
            blobs[k] = base.rve_save_state()
    rolled_back = failed = 0
    for k, blob in blobs.items():
        for mult in (1, 2, 4):
            for ms in (15, 25, 40):
                r = m.from_workload(w, max_stagger=ms, max_halvings=1)
                r.rve_load_state(blob)
                before = _snapshot(r)
                info, st = r.rve_run_slots([mult * w.dtau], [1])
                if st[0] != m.RVE_OK:
                    failed += 1
                    assert st[0] == m.RVE_ENOCONV and info[0]["reason"] == 1   # RVE_WHY_STAGGER
                    _same(before, _snapshot(r))
                    if info[0]["n_substeps"] > 0:
                        rolled_back += 1
                        print("rolled back: state", k, "dtau x", mult, "max_stagger", ms,
                              "sub-steps committed first", info[0]["n_substeps"], flush=True)
                else:
                    assert r.rve_get_scalars()["step"] == before[2]["step"] + info[0]["n_substeps"]
                r.close()
    print("failed calls", failed, "with a roll-back", rolled_back, flush=True)
    assert rolled_back > 0, "no case committed a sub-step before failing"


def test_non_finite_inputs_are_rejected():
    from paper_2508_07424_amd import mirve as m
    w = W.composite_2d_small()
    r = m.from_workload(w)
    before = _snapshot(r)
    for name in ("phi", "hist"):
        bad = before[0].copy()
        bad.flat[5] = np.nan
        with pytest.raises(m.MirveError) as e:
            r.rve_set_field(name, bad)
        assert e.value.code == m.RVE_EINVAL
    with pytest.raises(m.MirveError) as e:
        r.rve_step_dissipation(float("nan"))
    assert e.value.code == m.RVE_EINVAL
    with pytest.raises(m.MirveError) as e:
        r.rve_step_dissipation(float("inf"))
    assert e.value.code == m.RVE_EINVAL
    theta = np.zeros(w.shape)
    theta[3, 4] = np.inf
    with pytest.raises(m.MirveError) as e:
        r.rve_set_microstructure(w.phase_id, w.phases, theta=theta, void=w.void, phi_disc=w.phi_disc)
    assert e.value.code == m.RVE_EINVAL
    for key in ("E", "Gc"):
        ph = [dict(p) for p in w.phases]
        ph[0][key] = float("nan")
        with pytest.raises(m.MirveError) as e:
            r.rve_set_microstructure(w.phase_id, ph, void=w.void, phi_disc=w.phi_disc)
        assert e.value.code == m.RVE_EINVAL
    for beta in (float("nan"), -1.5):        # A_f = I + beta (I - n n) must stay positive
        ph = [dict(p) for p in w.phases]
        ph[1]["beta"] = beta
        with pytest.raises(m.MirveError) as e:
            r.rve_set_microstructure(w.phase_id, ph, void=w.void, phi_disc=w.phi_disc)
        assert e.value.code == m.RVE_EINVAL
    sc = dict(before[2])
    sc["E"] = float("nan")
    with pytest.raises(m.MirveError) as e:
        r.rve_set_scalars(sc)
    assert e.value.code == m.RVE_EINVAL
    # the rejected calls left the handle as it was (the microstructure calls
    # fail before they touch the slot's state)
    after = _snapshot(r)
    _same(before, after)
    r.rve_step_dissipation(w.dtau)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_checkpoint_resume_is_bitwise(prec):
    from paper_2508_07424_amd import mirve as m
    w = W.composite_2d_small()
    a = m.from_workload(w, precision=prec)
    for _ in range(3):
        a.rve_step_dissipation(w.dtau)
    blob = a.rve_save_state()
    b = m.from_workload(w, precision=prec)
    b.rve_load_state(blob)
    _same(_snapshot(a), _snapshot(b))
    for k in range(3):
        ia = a.rve_step_dissipation(w.dtau)
        ib = b.rve_step_dissipation(w.dtau)
        print("step", k + 4, ia["E"], ib["E"], flush=True)
        for key in ("E", "Sigma", "D", "T", "n_stagger", "n_cg", "n_pcg"):
            assert ia[key] == ib[key], (key, ia[key], ib[key])
    _same(_snapshot(a), _snapshot(b))
    # a blob of another grid is refused
    other = m.from_workload(W.homogeneous_2d(nx=32, ny=32, crack=8), precision=prec)
    with pytest.raises(m.MirveError) as e:
        other.rve_load_state(blob)
    assert e.value.code == m.RVE_EINVAL
