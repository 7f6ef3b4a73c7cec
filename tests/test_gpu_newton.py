"""The paper's monolithic per-step solver on the GPU (Sec. 4.1, Eq. 22-31):
Newton-Raphson on (eps~, phi, E) with the Jacobian applied through the
Green operator, the damage stencil and a reduction, each Newton system
solved by restarted GMRES, the relaxation of Eq. 31.

Against the oracle's Newton solver (stored run of 22 steps past the peak
load, where alpha < 1), against the staggered step on the GPU (the same
per-step fixed point), and the contract: a failed step leaves the state
bitwise unchanged, FP64 and the law without split only, slots of a batched
handle independent.
"""
import json
import os

import numpy as np
import pytest

from oracle import newton, solver
from paper_2508_07424_amd import workloads as W
from tests.helpers import oracle_problem, rel

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "newton_plate12_fp64.json")
TIGHT = dict(tol=1e-10, tol_cg=1e-12, tol_pcg=1e-14, tol_al=1e-12)


def _plate(**kw):
    from paper_2508_07424_amd import mirve as m
    w = W.two_phase_plate_2d()
    return w, m.from_workload(w, **dict(TIGHT, **kw))


def _state(r, slot=0):
    return (r.rve_get_field("phi", slot=slot), r.rve_get_field("hist", slot=slot),
            r.rve_get_scalars(slot=slot))


def test_newton_matches_the_stored_oracle_run():
    """22 Newton steps on the GPU against the oracle's Newton run: E, Sigma,
    D, T, Gamma per step and the final damage to 1e-10; the relaxation
    factor of Eq. 31 goes below 1 past the peak on both sides (the GPU
    reports no alpha; the steps past the peak agree only if it is the
    same)."""
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    w, r = _plate()
    assert abs(r.rve_get_scalars()["tau0"] - gold["tau0"]) <= 1e-12 * gold["tau0"]
    worst = 0.0
    for k, g in enumerate(gold["steps"]):
        info = r.rve_step_newton(w.dtau, tol=gold["newton_tol"], krylov_tol=gold["krylov_tol"])
        dev = max(abs(info[key] - g[key]) / abs(g[key]) for key in ("E", "Sigma", "D", "T", "Gamma"))
        worst = max(worst, dev)
        print("step", k + 1, "alpha %.6f" % g["alpha"], "newton", info["n_stagger"], "oracle", g["n_newton"],
              "gmres", info["n_cg"], "dev %.2e" % dev, flush=True)
        assert info["step"] == k + 1 and info["reason"] == 0
        assert dev <= 1e-10, (k + 1, {key: (info[key], g[key]) for key in ("E", "Sigma", "D", "T")})
    assert min(g["alpha"] for g in gold["steps"]) < 0.99
    assert rel(r.rve_get_field("phi").ravel(), np.asarray(gold["phi"])) <= 1e-10
    print("worst step deviation %.2e" % worst, flush=True)


def test_newton_and_staggered_reach_the_same_fixed_point():
    """Both GPU solvers on one notched plate, step for step (Sec. 4.1 against
    Eq. 16): E, Sigma, D, T and the damage agree to 1e-9; a Newton step can
    follow staggered steps on the same handle and the reverse, and the oracle
    doing the same sequence agrees."""
    from paper_2508_07424_amd import mirve as m
    w = W.homogeneous_2d(nx=24, ny=16, crack=6)
    a = m.from_workload(w, **TIGHT)
    b = m.from_workload(w, **TIGHT)
    prob = oracle_problem(w, tol=1e-11, tol_cg=1e-13, tol_al=1e-13)
    st = solver.State(prob)
    plan = ["newton", "newton", "staggered", "newton", "staggered", "staggered"]
    for k, how in enumerate(plan):
        ia = a.rve_step_dissipation(w.dtau)
        ib = b.rve_step_newton(w.dtau, tol=1e-11) if how == "newton" else b.rve_step_dissipation(w.dtau)
        ro = newton.step(prob, st, w.dtau, tol=1e-11) if how == "newton" else solver.step(prob, st, w.dtau)
        for key in ("E", "Sigma", "D", "T"):
            assert abs(ia[key] - ib[key]) <= 1e-9 * abs(ia[key]), (k, how, key, ia[key], ib[key])
            assert abs(ib[key] - ro[key]) <= 1e-9 * abs(ro[key]), (k, how, key, ib[key], ro[key])
        print("step", k + 1, how, "E", ib["E"], "newton iterations", ib["n_stagger"], flush=True)
    assert rel(a.rve_get_field("phi"), b.rve_get_field("phi")) <= 1e-9
    assert rel(b.rve_get_field("phi"), prob.to_public(st.phi)) <= 1e-9


def test_failed_newton_step_leaves_the_state_unchanged():
    """max_newton = 1 cannot meet Eq. 30 from a fresh step: RVE_ENOCONV
    with reason RVE_WHY_NEWTON, fields and scalars bitwise as before; the
    same handle then takes the step with the defaults."""
    from paper_2508_07424_amd import mirve as m
    w, r = _plate()
    r.rve_step_newton(w.dtau)
    before = _state(r)
    with pytest.raises(m.MirveError) as e:
        r.rve_step_newton(w.dtau, max_newton=1)
    assert e.value.code == m.RVE_ENOCONV
    after = _state(r)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert before[2] == after[2]
    info = r.rve_step_newton(w.dtau)
    assert info["step"] == 2


def test_newton_rejects_what_it_does_not_cover():
    from paper_2508_07424_amd import mirve as m
    w = W.two_phase_plate_2d()
    mixed = m.from_workload(w, precision=m.RVE_PREC_MIXED)
    with pytest.raises(m.MirveError) as e:
        mixed.rve_step_newton(w.dtau)
    assert e.value.code == m.RVE_EINVAL
    split = m.from_workload(w, split=m.RVE_SPLIT_VOLDEV)
    with pytest.raises(m.MirveError) as e:
        split.rve_step_newton(w.dtau)
    assert e.value.code == m.RVE_EINVAL
    _, r = _plate()
    for bad in (dict(restart=0), dict(krylov_tol=0.0), dict(theta=0.0), dict(max_newton=0)):
        with pytest.raises(m.MirveError) as e:
            r.rve_step_newton(w.dtau, **bad)
        assert e.value.code == m.RVE_EINVAL, bad
    with pytest.raises(m.MirveError) as e:
        r.rve_step_newton(float("nan"))
    assert e.value.code == m.RVE_EINVAL
    assert r.rve_get_scalars()["step"] == 0


def test_newton_on_a_slot_of_a_batch_equals_alone():
    """A Newton step on slot 1 of a two-slot handle gives bitwise the step
    of the same RVE alone, and leaves slot 0 as it was."""
    from paper_2508_07424_amd import mirve as m
    w = W.two_phase_plate_2d()
    w2 = W.two_phase_plate_2d(seed=5)
    batch = m.from_workloads([w2, w], **TIGHT)
    alone = m.from_workload(w, max_materials=batch.cfg.max_materials, **TIGHT)
    before0 = _state(batch, 0)
    for _ in range(2):
        ib = batch.rve_step_newton(w.dtau, slot=1)
        ia = alone.rve_step_newton(w.dtau)
        for key in ("E", "Sigma", "D", "T", "Gamma", "n_stagger", "n_cg"):
            assert ib[key] == ia[key], (key, ib[key], ia[key])
    assert np.array_equal(batch.rve_get_field("phi", slot=1), alone.rve_get_field("phi"))
    after0 = _state(batch, 0)
    assert np.array_equal(before0[0], after0[0]) and before0[2] == after0[2]


def test_newton_3d_matches_the_oracle_newton():
    """The 3D form (s = 6, the Green operator's z pass) on an 8 x 6 x 6
    two-phase RVE with a square notch, loaded along z: three Newton steps
    against the oracle's Newton steps to 1e-10."""
    from paper_2508_07424_amd import mirve as m
    n = (8, 6, 6)
    rng = np.random.default_rng(9)
    pid = (rng.random((6, 6, 8)) < 0.4).astype(np.uint16)
    void, tips = W.notch_3d_square(n, 1.0, 3, 2, 6, 2, 4)
    pid[void.astype(bool)] = 0
    w = W.Workload(n=n, h=1.0, ell=1.5, phases=[W.iso(1, 0.3, 1), W.iso(3, 0.25, 2)], phase_id=pid,
                   f=W.load_zz(), dtau=0.3, void=void, phi_disc=tips)
    r = m.from_workload(w, **TIGHT)
    prob = oracle_problem(w, tol=1e-11, tol_cg=1e-12, tol_al=1e-12)
    st = solver.State(prob)
    for k in range(3):
        info = r.rve_step_newton(w.dtau, tol=1e-11)
        rec = newton.step(prob, st, w.dtau, tol=1e-11)
        dev = max(abs(info[key] - rec[key]) / abs(rec[key]) for key in ("E", "Sigma", "D", "T", "Gamma"))
        print("step", k + 1, "newton", info["n_stagger"], "oracle", rec["n_newton"], "dev %.2e" % dev, flush=True)
        assert dev <= 1e-10
    assert rel(r.rve_get_field("phi"), prob.to_public(st.phi)) <= 1e-10
