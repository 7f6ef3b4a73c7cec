"""The paper's monolithic per-step solver (Sec. 4.1, Eq. 22-31): Newton-Raphson
on q = (eps~, phi, E), each Newton system solved by a Krylov method.

Oracle; test infrastructure only.  Plain NumPy/SciPy, FP64.  It reaches the
same per-step fixed point as the staggered solver of solver.py (R1 = R2 =
R3 = 0 with the history of Eq. 38), by another route.

Readings (the same as the staggered oracle where they overlap):
* R1 carries g(phi) (Eq. 29: C_i = C(q_i)); the projection is the symmetric
  P of spectral.py (Eq. 26).
* H_i = max(psi_o(eps_i) + psi_ini, H^n) (Eq. 38 with the enrichment energy).
  Eq. 27 compares psi_o with H_i itself, which the max never exceeds; the
  Jacobian takes dH/deps = sigma_o where psi_o + psi_ini >= H^n and psi_o > 0
  (non-strict: at the start of a step the loaded region sits exactly at
  H^n, and a strict test would leave the Jacobian singular in E), 0 on notch
  voxels (no driving force there).  The residual uses the max itself, so the
  fixed point is the staggered solver's.
* At E = 0 the Jacobian is singular (D does not depend on E to first
  order), so a step from the unloaded state starts from the elastic
  unit-load solution scaled to the staggered solver's first guess
  E = sqrt(min G_c / (l max psi_o1)).
* J3 is dD/dphi . dphi = int G_c (phi dphi / l + l grad phi . A grad dphi)
  with G_c inside the divergence (reading of the printed J3).
* Convergence (Eq. 30): max(||dE_total||/||eps||, ||dphi||/||phi||,
  |D - tau|/tau) < tol, with the absolute value on the last term.
* Relaxation (Eq. 31): the printed ratio is always >= 1; it is read as
  alpha^n = max(theta, Sigma^(n-1) / max_(j<n) Sigma^j), theta = 0.3, so
  that alpha = 1 until the load drops and then decreases.  With
  relax=False every Newton step is taken in full.
* The linear system is non-symmetric (the g' couplings and dH/deps) and,
  on the full strain space, singular: J1 sees only the compatible part of a
  strain.  The operator handed to the Krylov solver is J on the compatible
  part plus the identity on the incompatible part (P dx is used, and
  (I - P) dx is returned as it is), which is non-singular and whose
  solution for the (compatible) right-hand side is compatible.  The paper
  names BiCGSTAB; on this operator it diverged or lost its residual
  (tested on 12 x 8 and 24 x 16 plates), so the oracle takes restarted
  GMRES (scipy.sparse.linalg.gmres), a library solver of the same system:
  the Newton iterates and the fixed point do not depend on which Krylov
  method solves it to the tolerance.
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

from . import model, solver, spectral


class NewtonNotConverged(RuntimeError):
    pass


def _fields(prob, st, x, E):
    """Total strain, undegraded stress and energy, history and its active set."""
    eps = x + E * prob.f.reshape((-1,) + (1,) * prob.d)
    sig0 = model.stress_undegraded(eps, prob.mat)
    psi0 = np.where(prob.mat.void, 0.0, 0.5 * np.sum(eps * sig0, axis=0))
    ht = psi0 + st.psi_ini
    H = np.maximum(ht, st.H) if prob.history else ht
    active = (ht >= st.H) if prob.history else np.ones(prob.n, dtype=bool)
    active = active & ~prob.mat.void & (psi0 > 0.0)
    return eps, sig0, H, active


def residual(prob, st, x, phi, E, tau):
    """R1, R2, R3 of Eq. 24 at q = (x, phi, E)."""
    eps, sig0, H, _ = _fields(prob, st, x, E)
    g = model.degradation(phi, prob.k)
    R1 = spectral.green_apply(g * sig0, prob.P)
    A = prob.mat.A
    R2 = (prob.mat.Gc / prob.ell + 2.0 * H) * phi - 2.0 * H + \
        model.damage_operator(phi, prob.mat.Gc, prob.ell, prob.h, A)
    R3 = model.dissipation(phi, prob.mat.Gc, prob.ell, prob.h, A) - tau
    return R1, R2, R3


def jacobian_apply(prob, st, x, phi, E, dx, dphi, dE):
    """J1, J2, J3 of Eq. 25 applied to dq = (dx, dphi, dE)."""
    eps, sig0, H, active = _fields(prob, st, x, E)
    g = model.degradation(phi, prob.k)
    gp = -2.0 * (1.0 - phi)
    de = dx + dE * prob.f.reshape((-1,) + (1,) * prob.d)
    J1 = spectral.green_apply(g * model.stress_undegraded(de, prob.mat) + gp * sig0 * dphi, prob.P)
    dH = np.where(active, np.sum(sig0 * de, axis=0), 0.0)
    A = prob.mat.A
    J2 = gp * dH + (prob.mat.Gc / prob.ell + 2.0 * H) * dphi + \
        model.damage_operator(dphi, prob.mat.Gc, prob.ell, prob.h, A)
    dens = prob.mat.Gc * phi * dphi / prob.ell
    for j in range(prob.d):
        for k in range(prob.d):
            if A is None and j != k:
                continue
            a = 1.0 if A is None else A[..., j, k]
            dens = dens + prob.mat.Gc * prob.ell * a * model.forward_difference(phi, j, prob.h) * \
                model.forward_difference(dphi, k, prob.h)
    J3 = float(np.sum(dens) * prob.h ** prob.d)
    return J1, J2, J3


def step(prob, st, dtau, tol=None, max_newton=50, krylov_tol=1e-12, relax=True, theta=0.3,
         restart=200):
    """One dissipation-controlled step tau^(n+1) = tau^n + dtau by Newton-Raphson
    (Eq. 22-31).  Updates st like solver.step and returns its record; raises
    NewtonNotConverged (state unchanged) if Newton does not converge."""
    tol = prob.tol if tol is None else tol
    tau = st.tau + dtau
    # the state keeps the unit-load fluctuation (eps = E (f + x)); Newton works
    # on the fluctuation of the actual strain, E x
    x, phi, E = st.E * st.x, st.phi.copy(), st.E
    if E == 0.0:
        x1, _ = solver.mechanics(prob, phi, st.x)
        _, _, psi1, _ = solver.unit_response(prob, phi, x1)
        pmax = float(np.max(psi1))
        E = math.sqrt(float(np.min(prob.mat.Gc)) / prob.ell / pmax) if pmax > 0 else 1.0
        x = E * x1
    s, n = prob.s, prob.n
    N = int(np.prod(n))
    size = (s + 1) * N + 1
    # relaxation of Eq. 31 (reading in the module docstring)
    alpha = 1.0
    if relax and len(st.curve) > 2:
        sig_prev = st.curve[-1]["Sigma"]
        sig_max = max(r["Sigma"] for r in st.curve[:-1])
        if sig_max > 0.0:
            alpha = max(theta, min(1.0, sig_prev / sig_max))

    def pack(a, b, c):
        return np.concatenate([a.ravel(), b.ravel(), [c]])

    def unpack(v):
        return v[: s * N].reshape((s,) + n), v[s * N: (s + 1) * N].reshape(n), v[-1]

    n_krylov = 0
    for it in range(1, max_newton + 1):
        R1, R2, R3 = residual(prob, st, x, phi, E, tau)

        def mv(v):
            # J on the compatible part of the strain, identity on the rest
            dx, dphi, dE = unpack(v)
            pdx = spectral.green_apply(dx, prob.P)
            J1, J2, J3 = jacobian_apply(prob, st, x, phi, E, pdx, dphi, dE)
            return pack(J1 + (dx - pdx), J2, J3)

        J = spla.LinearOperator((size, size), matvec=mv, dtype=float)
        rhs = -pack(R1, R2, R3)
        counter = {"n": 0}

        def cb(_):
            counter["n"] += 1
        sol, info = spla.gmres(J, rhs, rtol=krylov_tol, atol=0.0, restart=restart, maxiter=100,
                               callback=cb, callback_type="pr_norm")
        n_krylov += counter["n"]
        if info != 0:
            raise NewtonNotConverged("GMRES did not converge (info=%d)" % info)
        dx, dphi, dE = unpack(sol)
        dx = spectral.green_apply(dx, prob.P)
        x = x + alpha * dx
        phi = phi + alpha * dphi
        E = E + alpha * dE
        eps = x + E * prob.f.reshape((-1,) + (1,) * prob.d)
        de = dx + dE * prob.f.reshape((-1,) + (1,) * prob.d)
        D = model.dissipation(phi, prob.mat.Gc, prob.ell, prob.h, prob.mat.A)
        err = max(math.sqrt(np.sum(de * de)) / max(math.sqrt(np.sum(eps * eps)), 1e-300),
                  math.sqrt(np.sum(dphi * dphi)) / max(math.sqrt(np.sum(phi * phi)), 1e-300),
                  abs(D - tau) / tau)
        if err < tol:
            break
    else:
        raise NewtonNotConverged("Newton did not converge (err=%g)" % err)
    # commit: history, curve (Eq. 33, 38)
    _, sig0, H, _ = _fields(prob, st, x, E)
    g = model.degradation(phi, prob.k)
    Sigma = float(np.sum(np.mean((g * sig0).reshape(s, -1), axis=1) * prob.f))
    st.T += 0.5 * (Sigma + st.Sigma) * (E - st.E)
    st.phi, st.E, st.H, st.Sigma, st.tau = phi, E, H, Sigma, tau
    st.x = x / E if E != 0.0 else np.zeros_like(x)
    st.step += 1
    st.fractured = solver.fractured(prob, phi)
    rec = dict(step=st.step, E=E, Sigma=Sigma, T=st.T, D=D,
               Gamma=model.crack_surface(phi, prob.ell, prob.h, prob.mat.A), tau=tau,
               n_newton=it, n_krylov=n_krylov, alpha=alpha, fractured=st.fractured)
    rec["G_inst"] = solver.instantaneous_G(prob, st.curve[-1], rec)
    st.curve.append(rec)
    return rec
