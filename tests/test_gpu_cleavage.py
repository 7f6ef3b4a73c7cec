"""Cleavage anisotropy on the GPU against the oracle (Sec. 2.2, Eq. 14-17;
the enrichment with the cleavage tensor, Eq. 36-37b).

Phases carry a weak-plane normal rotated with the voxel's angle and a weight
beta; the damage operator, D and Gamma, the tangent dD/dE and the
enrichment use A = I + beta (I - n n).  FP64 results agree with the oracle
to 1e-10 (initial state, damage solve, steps), as for isotropic phases.
"""
import numpy as np
import pytest

from oracle import model, solver
from paper_2508_07424_amd import workloads as W
from tests.helpers import oracle_problem, rel

pytestmark = pytest.mark.gpu

TIGHT = dict(tol=1e-12, tol_cg=1e-13, tol_pcg=1e-14, tol_al=1e-13)
OTIGHT = dict(tol=1e-12, tol_cg=1e-13, tol_al=1e-13)


def _poly(n=40, beta=2.0, seed=7):
    return W.polycrystal_2d(n=n, grains=8, seed=seed, zener=2.0, a_cleave=1.0, beta=beta)


def _plate3d():
    """12 x 10 x 14 two-phase 3D RVE with rotated cleavage normals and a
    square notch in the z mid-plane."""
    n = (12, 10, 14)
    rng = np.random.default_rng(9)
    shape = tuple(reversed(n))
    pid = (rng.random(shape) < 0.4).astype(np.uint16)
    theta = rng.uniform(0.0, np.pi, size=shape)
    phases = [dict(W.iso(1.0, 0.3, 1.0), beta=1.5, n=(0.0, 0.6, 0.8)),
              dict(W.cubic(3.0, 1.2, 0.9, 2.0), beta=3.0, n=(1.0, 0.0, 0.0))]
    void, tips = W.notch_3d_square(n, 1.0, 7, 3, 8, 3, 7)
    pid[void.astype(bool)] = 0
    return W.Workload(n=n, h=1.0, ell=1.5, phases=phases, phase_id=pid, f=W.load_zz(), dtau=1.0,
                      theta=theta, void=void, phi_disc=tips, phi_M=0.8)


CASES = [("poly40-beta2", lambda: _poly()), ("plate3d", _plate3d)]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_cleavage_initial_state(name, make):
    from paper_2508_07424_amd import mirve as m
    w = make()
    print("case", name, w.n, flush=True)
    r = m.from_workload(w)
    prob = oracle_problem(w)
    assert prob.mat.A is not None
    st = solver.State(prob)
    e1 = rel(r.rve_get_field("phi_ini"), prob.to_public(st.phi_ini))
    e2 = rel(r.rve_get_field("psi_ini"), prob.to_public(st.psi_ini))
    tau0 = r.rve_get_scalars()["tau0"]
    print("phi_ini %.3e psi_ini %.3e tau0 %.3e" % (e1, e2, abs(tau0 - st.tau) / st.tau), flush=True)
    assert e1 < 1e-11 and e2 < 1e-9
    assert abs(tau0 - st.tau) <= 1e-11 * st.tau


@pytest.mark.parametrize("pre", [0, 1], ids=["fft", "jacobi"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_cleavage_damage_solve(name, make, pre):
    from paper_2508_07424_amd import mirve as m
    w = make()
    r = m.from_workload(w, damage_precond=pre, **TIGHT)
    prob = oracle_problem(w, **OTIGHT)
    st = solver.State(prob)
    x, _ = solver.mechanics(prob, st.phi, st.x)
    _, _, psi1_o, _ = solver.unit_response(prob, st.phi, x)
    r.rve_set_field("psi1", prob.to_public(psi1_o))
    E = 1.5 * np.sqrt(1.0 / prob.ell / max(psi1_o.max(), 1e-300))
    D, npcg = r.rve_solve_damage(E, commit=True)
    H = solver.history_field(prob, E, psi1_o, st.psi_ini, st.H)
    phi_o = model.solve_damage(H, prob.mat.Gc, prob.ell, prob.Dmats, A=prob.mat.A)
    D_o = model.dissipation(phi_o, prob.mat.Gc, prob.ell, prob.h, prob.mat.A)
    e = rel(r.rve_get_field("phi"), prob.to_public(phi_o))
    print("case", name, "pcg iterations", npcg, "D rel %.3e phi %.3e" % (abs(D - D_o) / D_o, e),
          flush=True)
    assert abs(D - D_o) <= 1e-10 * D_o
    assert e < 1e-10


def test_cleavage_steps_fp64():
    from paper_2508_07424_amd import mirve as m
    w = _poly(n=32, beta=3.0, seed=4)
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
    assert rel(r.rve_get_field("phi"), prob.to_public(st.phi)) < 1e-10
