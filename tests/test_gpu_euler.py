"""Grain orientations in three dimensions on the GPU (Sec. 5.3): z-x-z Euler
angles per voxel rotate the cubic stiffness and the cleavage normal; the
paper's one-voxel plates are grids of two identical layers along z.

FP64 results agree with the oracle to 1e-10 (initial state, Green operator,
steps), and a plate whose grains turn about z only is the 2D plane-strain
problem on the GPU as well.
"""
import numpy as np
import pytest

from oracle import solver, spectral, model
from paper_2508_07424_amd import workloads as W
from tests.helpers import oracle_problem, rel, to_oracle

pytestmark = pytest.mark.gpu

TIGHT = dict(tol=1e-12, tol_cg=1e-13, tol_pcg=1e-14, tol_al=1e-13)
OTIGHT = dict(tol=1e-12, tol_cg=1e-13, tol_al=1e-13)


def _plate():
    return W.polycrystal_plate(n=24, layers=2, grains=6, seed=11, zener=3.0, beta=1.5)


def test_plate_initial_state_and_operator():
    from paper_2508_07424_amd import mirve as m
    w = _plate()
    print("plate", w.n, "grains", w.meta["grains"], flush=True)
    r = m.from_workload(w, **TIGHT)
    prob = oracle_problem(w, **OTIGHT)
    assert prob.mat.A is not None
    st = solver.State(prob)
    assert rel(r.rve_get_field("phi_ini"), prob.to_public(st.phi_ini)) < 1e-11
    assert rel(r.rve_get_field("psi_ini"), prob.to_public(st.psi_ini)) < 1e-9
    assert abs(r.rve_get_scalars()["tau0"] - st.tau) <= 1e-11 * st.tau
    eps = np.random.default_rng(4).standard_normal((6,) + w.shape)
    gpu = r.rve_apply_green_op(eps)
    sig = model.stress(to_oracle(eps, 3), st.phi, prob.mat)
    ref = prob.to_public(spectral.green_apply(sig, prob.P))
    assert rel(gpu, ref) < 1e-12


def test_plate_steps_fp64():
    from paper_2508_07424_amd import mirve as m
    w = _plate()
    r = m.from_workload(w, **TIGHT)
    prob = oracle_problem(w, **OTIGHT)
    st = solver.State(prob)
    for k in range(3):
        info = r.rve_step_dissipation(w.dtau)
        rec = solver.step(prob, st, w.dtau)
        dev = {key: abs(info[key] - rec[key]) / abs(rec[key]) for key in ("E", "Sigma", "D", "T", "Gamma")}
        print("step", k + 1, dev, flush=True)
        for key, d in dev.items():
            assert d <= 1e-10, (key, info[key], rec[key])
    phi = r.rve_get_field("phi")
    assert rel(phi, prob.to_public(st.phi)) < 1e-10
    # the two layers carry the same damage
    assert np.array_equal(phi[0], phi[1])


def test_plate_turned_about_z_is_the_2d_problem():
    """Grains turned about z only: E and Sigma of the two-layer plate equal
    those of the 2D grid with the same in-plane angles, D twice the 2D one."""
    from paper_2508_07424_amd import mirve as m
    w2 = W.polycrystal_2d(n=32, grains=8, seed=5, zener=2.0, a_cleave=1.0, beta=2.0)
    rep = lambda a: np.ascontiguousarray(np.broadcast_to(a, (2,) + a.shape))
    eu = np.stack([w2.theta, np.zeros_like(w2.theta), np.zeros_like(w2.theta)], axis=-1)
    f = np.zeros(6)
    f[1] = 1.0
    w3 = W.Workload(n=w2.n + (2,), h=w2.h, ell=w2.ell, phases=w2.phases, phase_id=rep(w2.phase_id), f=f,
                    dtau=2 * w2.dtau, void=rep(w2.void), phi_disc=rep(w2.phi_disc), phi_M=w2.phi_M,
                    euler=rep(eu))
    r2 = m.from_workload(w2, **TIGHT)
    r3 = m.from_workload(w3, **TIGHT)
    for k in range(3):
        a = r2.rve_step_dissipation(w2.dtau)
        b = r3.rve_step_dissipation(w3.dtau)
        print("step", k + 1, a["E"], b["E"], flush=True)
        for key in ("E", "Sigma"):
            assert abs(a[key] - b[key]) <= 1e-9 * abs(a[key]), (key, a[key], b[key])
        assert abs(2 * a["D"] - b["D"]) <= 1e-9 * abs(b["D"])


def test_euler_input_is_checked():
    from paper_2508_07424_amd import mirve as m
    w = _plate()
    r = m.from_workload(w)
    bad = w.euler.copy()
    bad[0, 3, 4, 1] = np.inf
    with pytest.raises(m.MirveError) as e:
        r.rve_set_microstructure_euler(w.phase_id, w.phases, bad, void=w.void, phi_disc=w.phi_disc)
    assert e.value.code == m.RVE_EINVAL
    assert r.rve_get_scalars()["step"] == 0


def test_euler_on_a_2d_grid():
    """A 2D (plane-strain) grid takes the in-plane block of the stiffness and
    of the cleavage tensor rotated by general Euler angles: the Green
    operator, the initial state and two steps against the oracle."""
    from paper_2508_07424_amd import mirve as m
    w = W.polycrystal_2d(n=32, grains=8, seed=6, zener=3.0, a_cleave=1.0, beta=2.0)
    rng = np.random.default_rng(2)
    ang = np.stack([rng.uniform(0, 2 * np.pi, 8), np.arccos(rng.uniform(-1, 1, 8)),
                    rng.uniform(0, 2 * np.pi, 8)], axis=-1)
    w.euler = ang[w.phase_id]
    w.theta = None
    r = m.from_workload(w, **TIGHT)
    prob = oracle_problem(w, **OTIGHT)
    st = solver.State(prob)
    eps = np.random.default_rng(5).standard_normal((3,) + w.shape)
    sig = model.stress(to_oracle(eps, 2), st.phi, prob.mat)
    assert rel(r.rve_apply_green_op(eps), prob.to_public(spectral.green_apply(sig, prob.P))) < 1e-12
    assert rel(r.rve_get_field("phi_ini"), prob.to_public(st.phi_ini)) < 1e-11
    for k in range(2):
        info = r.rve_step_dissipation(w.dtau)
        rec = solver.step(prob, st, w.dtau)
        for key in ("E", "Sigma", "D", "T"):
            assert abs(info[key] - rec[key]) <= 1e-10 * abs(rec[key]), (k, key)
