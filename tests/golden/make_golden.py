"""Write the stored full-run results of the oracle (run from the repository
root: python tests/golden/make_golden.py).  Only oracle/ and the geometry
generators are used.

homogeneous32_fp64.json: a homogeneous plate broken in two, run to the
fracture point; per step E, Sigma, D, T and G_eff (Eq. 32-33).
composite64_fp64.json: the first 60 steps of the 64 x 64 composite.
sampling24_fp64.json: the toughness of a 24 x 24 plate with one inclusion
at four initial-crack positions and their minimum (Sec. 3).
newton_plate12_fp64.json: 22 steps of the monolithic Newton-Raphson solver
(Sec. 4.1) on a 12 x 10 two-phase plate, past the peak load.
Both with tight tolerances (stagger 1e-10, Krylov and constraint 1e-12).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solver  # noqa: E402
from paper_2508_07424_amd import workloads as W  # noqa: E402

TOL = dict(tol=1e-10, tol_cg=1e-12, tol_al=1e-12, max_stagger=300)


def _record(rec):
    return {k: (float(v) if not isinstance(v, bool) else v) for k, v in rec.items()}


def _problem(w):
    return solver.Problem(w.n, w.h, w.ell, w.phases, w.phase_id, w.f, theta=w.theta, void=w.void,
                          phi_disc=w.phi_disc, phi_M=w.phi_M, k=w.k, **TOL)


def homogeneous32():
    """Homogeneous 32 x 32 plate with an 8-voxel notch, run to the fracture
    point: the full curve and G_eff (Eq. 32-33)."""
    w = W.homogeneous_2d(nx=32, ny=32, crack=8)
    prob = _problem(w)
    t0 = time.time()
    curve = []

    def keep(rec):
        curve.append(_record(rec))
        print("homogeneous step", len(curve), "E %.6g Sigma %.6g stagger %d"
              % (rec["E"], rec["Sigma"], rec["n_stagger"]), flush=True)
    st, G = solver.run(prob, w.dtau, max_steps=400, callback=keep)
    return {"workload": "homogeneous_2d(nx=32, ny=32, crack=8)", "tolerances": TOL,
            "dtau": w.dtau, "A_g": prob.A_g, "V": prob.V, "tau0": float(st.tau0),
            "steps": curve, "G_eff": G, "seconds": round(time.time() - t0, 1)}


def composite64(nsteps=60):
    """The 64 x 64 two-phase composite (10 disks, 16-voxel notch, l = 1.5,
    dtau = 0.01 Gc L_x): the first nsteps steps.  Later, around step 68,
    the crack advances unstably and the staggered fixed point becomes too
    slow to reproduce step by step, so the stored curve stops before."""
    w = W.composite_2d_small()
    prob = _problem(w)
    st = solver.State(prob)
    t0 = time.time()
    curve = []
    for k in range(nsteps):
        rec = solver.step(prob, st, w.dtau)
        curve.append(_record(rec))
        print("composite step", k + 1, "E %.6g stagger %d" % (rec["E"], rec["n_stagger"]),
              flush=True)
    return {"workload": "composite_2d_small(seed=1)", "tolerances": TOL, "dtau": w.dtau,
            "tau0": float(st.tau0), "steps": curve, "seconds": round(time.time() - t0, 1)}


def sampling24(count=4):
    """Crack-position sampling (Sec. 3): the 24 x 24 plate with one disk
    inclusion, its microstructure shifted by 0, 6, 12, 18 voxels along the
    load axis, each run to its fracture point; G_eff per position and the
    minimum."""
    w = W.inclusion_2d()
    t0 = time.time()
    runs = []
    for sh, ws in W.crack_position_samples(w, count):
        prob = _problem(ws)
        st, G = solver.run(prob, ws.dtau, max_steps=400)
        runs.append({"shift": sh, "steps": st.step, "G_eff": G,
                     "G_inst": [r.get("G_inst") for r in st.curve[1:]]})
        print("sampling shift", sh, "steps", st.step, "G_eff", G, flush=True)
    g_min = min(r["G_eff"] for r in runs)
    return {"workload": "inclusion_2d() at %d crack positions" % count, "tolerances": TOL,
            "runs": runs, "G_min": g_min,
            "shift_min": [r["shift"] for r in runs if r["G_eff"] == g_min][0],
            "seconds": round(time.time() - t0, 1)}


def newton_plate12(nsteps=22):
    """The paper's monolithic Newton-Raphson step (Sec. 4.1, Eq. 22-31) on
    the 12 x 10 two-phase plate: nsteps steps, the last ones past the peak
    load, where the relaxation of Eq. 31 takes alpha < 1.  Newton tolerance
    1e-11, GMRES relative residual 1e-12."""
    from oracle import newton
    w = W.two_phase_plate_2d()
    prob = _problem(w)
    st = solver.State(prob)
    t0 = time.time()
    curve = []
    for k in range(nsteps):
        rec = newton.step(prob, st, w.dtau, tol=1e-11)
        curve.append(_record(rec))
        print("newton step", k + 1, "E %.6g alpha %.6g newton %d" % (rec["E"], rec["alpha"], rec["n_newton"]),
              flush=True)
    return {"workload": "two_phase_plate_2d()", "tolerances": TOL, "newton_tol": 1e-11,
            "krylov_tol": 1e-12, "dtau": w.dtau, "tau0": float(st.tau0), "steps": curve,
            "phi": st.phi.T.ravel().tolist(), "seconds": round(time.time() - t0, 1)}


if __name__ == "__main__":
    which = sys.argv[1:] or ["homogeneous32", "composite64", "sampling24", "newton_plate12"]
    for name in which:
        out = globals()[name]()
        path = os.path.join(ROOT, "tests", "golden", name + "_fp64.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", path, "steps", len(out.get("steps", out.get("runs", []))), "G_eff",
              out.get("G_eff", out.get("G_min")), flush=True)
