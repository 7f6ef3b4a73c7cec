"""Dissipation-controlled staggered solver and effective toughness (oracle).

TEST INFRASTRUCTURE ONLY.

The per-step problem is the fixed point of Eq. 16 (equilibrium, damage
balance with history, dissipation constraint) for the unknowns
{eps~, phi, E} with E_M = f E (Eq. 9).  The paper solves it monolithically
(Eq. 22-31); this oracle follows the staggered reading of the same fixed
point:

  (M)  equilibrium at fixed phi for a unit macroscopic load: the
       compatible, mean-free eps~_1 with P[sigma(f + eps~_1)] = 0
       (Fourier-Galerkin, Eq. 24 R1 / Eq. 26), by conjugate gradients.
       The stress is positively homogeneous of degree one in the strain,
       so eps = E (f + eps~_1) and psi_o = E^2 psi_o1.
  (A)  the scalar E >= 0 with D(phi(E)) = tau (Eq. 16c), where phi(E)
       solves the damage balance (Eq. 16b) with
       H(E) = max(E^2 psi_o1 + psi_ini, H^n) (Eq. 38; Eq. 11 history),
       found by safeguarded Newton; dD/dE comes from the tangent system.
  (U)  repeat (M), (A) until the changes of phi and E fall below tol
       (the relative-change test of Eq. 30).

The committed step stores phi, E, H^{n+1} = max(E^2 psi_o1 + psi_ini, H^n)
(Eq. 38 with psi_o1 of a final (M) at the committed phi), the macroscopic
stress Sigma = <sigma>:f and the running trapezoid T of Eq. 33.

Readings of the paper taken here: the fracture point
F (Sec. 4.2) is the first step at which every line of voxels along the
loading axis holds a broken voxel (phi >= 0.95, or a notch voxel);
A_g = h^(d-1) x (number of such lines without a notch voxel); V = N h^d;
tau^0 = D(phi_ini); the trapezoid of Eq. 33 is used (the text says Simpson,
the printed formula is the trapezoid).

Parity unpinned: the absolute effective toughness of a heterogeneous
composite or polycrystal.  It has no closed form and the paper's ensembles
are not given; the homogeneous, laminate and energy-balance cases pin the
steps it is made of, but the value itself is checked only against the HIP
path.
"""
import copy
import math
import numpy as np

from . import mandel, model, spectral


class Problem:
    """A periodic RVE toughness problem.

    Array inputs use the public layout: numpy arrays of shape reversed(n),
    i.e. (n_y, n_x) or (n_z, n_y, n_x) with x fastest.  They are transposed
    once here to the oracle's [x, y, z] indexing.
    """

    def __init__(self, n, h, ell, phases, phase_id, f, *, theta=None, void=None,
                 phi_disc=None, phi_M=0.8, k=1e-6, split="none", history=True,
                 A_g=None, tol=1e-10, tol_cg=1e-12, tol_al=1e-12, max_stagger=300,
                 max_cg=20000, frac_threshold=0.95, anderson_depth=5, max_halvings=8,
                 stall_window=0, euler=None):
        self.n = tuple(int(v) for v in n)
        self.d = len(self.n)
        self.s = mandel.nsym(self.d)
        self.h, self.ell, self.k = float(h), float(ell), float(k)
        self.split, self.history = split, bool(history)
        self.tol, self.tol_cg, self.tol_al = tol, tol_cg, tol_al
        self.max_stagger, self.max_cg = max_stagger, max_cg
        self.frac_threshold = frac_threshold
        self.anderson_depth = int(anderson_depth)
        self.max_halvings = int(max_halvings)
        self.stall_window = int(stall_window)
        tr = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a).T)
        pid = tr(phase_id)
        void_x = tr(void) if void is not None else np.zeros(self.n, dtype=bool)
        eu = None if euler is None else np.ascontiguousarray(
            np.moveaxis(np.asarray(euler, dtype=float), -1, 0).T)
        self.mat = model.MaterialField(self.n, phases, pid, theta=tr(theta), void=void_x, k=k,
                                       euler=eu)
        self.f = np.asarray(f, dtype=float)
        assert self.f.shape == (self.s,)
        self.load_axis = int(np.argmax(np.abs(self.f[: self.d])))
        self.P = spectral.projection_matrices(self.n, self.h)
        self.Dmats = model.difference_matrices(self.n, self.h)
        self.phi_disc = tr(phi_disc) if phi_disc is not None else np.zeros(self.n)
        self.phi_M = float(phi_M)
        self.V = float(np.prod(self.n)) * self.h ** self.d
        if A_g is None:
            broken_lines = np.any(self.mat.void, axis=self.load_axis)
            A_g = float(np.sum(~broken_lines)) * self.h ** (self.d - 1)
        self.A_g = float(A_g)

    # -- public-layout helper ---------------------------------------------
    def to_public(self, a):
        """[x, y, z] indexed field (optionally with a leading component axis)
        -> public layout (x fastest)."""
        if a.ndim == self.d:
            return np.ascontiguousarray(a.T)
        return np.ascontiguousarray(a.transpose((0,) + tuple(range(a.ndim - 1, 0, -1))))


# --------------------------------------------------------------------------
# (M) equilibrium at fixed damage
# --------------------------------------------------------------------------

def _dot(a, b):
    return float(np.sum(a * b))


def _uniform(f, n):
    return np.broadcast_to(f.reshape((-1,) + (1,) * len(n)), (f.size,) + tuple(n)).copy()


def mechanics(prob, phi, x0):
    """Equilibrium for the unit load f at damage phi (Eq. 16a, Eq. 24 R1).

    Returns (eps_tilde_1, iterations).  Conjugate gradients on the
    compatible subspace: A x = P[sigma(x)] is self-adjoint and positive on
    range(P) for the linear law.  With the volumetric split the law is
    piecewise linear and Newton iterations with the tangent stiffness are
    wrapped around the same CG.  The paper gives no solver for the split;
    here each tangent solve stops at ||r|| <= tol_cg ||P[sigma(f)]||, the
    load scale that ||b|| is for the linear law (a tolerance relative to the
    shrinking Newton residual would ask for accuracy below the rounding of
    the Green operator in the last Newton steps).
    """
    fU = _uniform(prob.f, prob.n)
    if prob.split == "none":
        x, it = _cg_linear(prob, phi, fU, x0, tangent=None)
        return x, it
    sf = spectral.green_apply(model.stress(fU, phi, prob.mat, prob.split), prob.P)
    r_abs = prob.tol_cg * math.sqrt(_dot(sf, sf))
    x = x0.copy()
    total = 0
    for _ in range(100):
        eps = fU + x
        R = -spectral.green_apply(model.stress(eps, phi, prob.mat, prob.split), prob.P)
        tr = eps[0] + eps[1] + (eps[2] if prob.d == 3 else 0.0)
        dx, it = _cg_tangent(prob, phi, tr, R, r_abs)
        total += it
        x = x + dx
        if math.sqrt(_dot(dx, dx)) <= prob.tol_cg * max(math.sqrt(_dot(x + fU, x + fU)), 1e-300):
            break
    return x, total


def _cg_linear(prob, phi, fU, x0, tangent=None):
    g = model.degradation(phi, prob.k)
    A = lambda v: spectral.green_apply(g * model.stress_undegraded(v, prob.mat), prob.P)
    b = -A(fU)
    x = x0.copy()
    r = b - A(x)
    bn = math.sqrt(_dot(b, b))
    if bn == 0.0:
        return np.zeros_like(x0), 0
    p = r.copy()
    rr = _dot(r, r)
    it = 0
    while math.sqrt(rr) > prob.tol_cg * bn and it < prob.max_cg:
        q = A(p)
        alpha = rr / _dot(p, q)
        x += alpha * p
        r -= alpha * q
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def _cg_tangent(prob, phi, tr, R, r_abs):
    """CG for P[C_t : dx] = R with the split's tangent stiffness, from
    dx = 0 until ||r|| <= r_abs."""
    g = model.degradation(phi, prob.k)
    I = model._identity(prob.d)
    Kb = prob.mat.K
    w = np.where(tr > 0, g, 1.0)

    def Ct(v):
        s0 = model.stress_undegraded(v, prob.mat)
        trv = v[0] + v[1] + (v[2] if prob.d == 3 else 0.0)
        out = np.empty_like(v)
        for a in range(prob.s):
            out[a] = g * (s0[a] - I[a] * Kb * trv) + w * I[a] * Kb * trv
        return out

    A = lambda v: spectral.green_apply(Ct(v), prob.P)
    x = np.zeros_like(R)
    r = R.copy()
    p = r.copy()
    rr = _dot(r, r)
    it = 0
    while math.sqrt(rr) > r_abs and it < prob.max_cg:
        q = A(p)
        alpha = rr / _dot(p, q)
        x += alpha * p
        r -= alpha * q
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def unit_response(prob, phi, x):
    """eps_1, psi_o1 and Sigma_1 = <sigma(eps_1)>:f for the unit load."""
    eps1 = _uniform(prob.f, prob.n) + x
    sig1 = model.stress(eps1, phi, prob.mat, prob.split)
    psi1 = model.energy_density(eps1, prob.mat, prob.split)
    Sigma1 = float(np.sum(np.mean(sig1.reshape(prob.s, -1), axis=1) * prob.f))
    return eps1, sig1, psi1, Sigma1


# --------------------------------------------------------------------------
# (A) dissipation constraint
# --------------------------------------------------------------------------

def history_field(prob, E, psi1, psi_ini, Hn):
    """H(E) = max(E^2 psi_o1 + psi_ini, H^n) (Eq. 38), or without the max."""
    Ht = E * E * psi1 + psi_ini
    return np.maximum(Ht, Hn) if prob.history else Ht


def arclength(prob, psi1, psi_ini, Hn, tau, E0):
    """Find E >= 0 with D(phi(E)) = tau (Eq. 16c) by safeguarded Newton.

    Returns (E, phi, number of damage solves)."""
    Gc, ell, h = prob.mat.Gc, prob.ell, prob.h
    nsolves = 0

    def evaluate(E):
        nonlocal nsolves
        H = history_field(prob, E, psi1, psi_ini, Hn)
        lu = model.factor_damage(H, Gc, ell, prob.Dmats, prob.mat.A)
        phi = lu.solve((2.0 * H).ravel()).reshape(prob.n)
        nsolves += 1
        return model.dissipation(phi, Gc, ell, h, prob.mat.A), phi, H, lu

    def derivative(E, phi, lu):
        Ht = E * E * psi1 + psi_ini
        active = (Ht > Hn) if prob.history else np.ones(prob.n, dtype=bool)
        dH = np.where(active, 2.0 * E * psi1, 0.0)
        dphi = lu.solve((2.0 * (1.0 - phi) * dH).ravel()).reshape(prob.n)
        # dD/dE = int G_c (phi phi' / l + l grad phi . A grad phi')
        A = prob.mat.A
        dens = Gc * phi * dphi / ell
        for j in range(prob.d):
            for k in range(prob.d):
                if A is None and j != k:
                    continue
                a = 1.0 if A is None else A[..., j, k]
                dens = dens + Gc * ell * a * model.forward_difference(phi, j, h) * \
                    model.forward_difference(dphi, k, h)
        return float(np.sum(dens) * h ** prob.d)

    lo, hi = 0.0, math.inf
    E = float(E0)
    if E <= 0.0:
        pmax = float(np.max(psi1))
        E = math.sqrt(float(np.min(Gc)) / ell / pmax) if pmax > 0 else 1.0
    for _ in range(200):
        Dv, phi, H, lu = evaluate(E)
        if abs(Dv - tau) <= prob.tol_al * tau:
            return E, phi, nsolves
        if Dv < tau:
            lo = max(lo, E)
        else:
            hi = min(hi, E)
        dD = derivative(E, phi, lu)
        En = E - (Dv - tau) / dD if dD > 0 else math.nan
        if not (lo < En < hi):
            En = 2.0 * E if math.isinf(hi) else 0.5 * (lo + hi)
        if not math.isinf(hi) and hi - lo <= 1e-15 * hi:
            return E, phi, nsolves
        E = En
    raise ConstraintNotConverged("arc-length root finder did not converge")


# --------------------------------------------------------------------------
# the step and the run
# --------------------------------------------------------------------------

class State:
    def __init__(self, prob):
        Gc = prob.mat.Gc
        A = prob.mat.A
        self.phi_ini = model.cte_initial_damage(prob.phi_disc, prob.ell, prob.h, prob.phi_M, A,
                                                prob.Dmats)
        self.psi_ini = model.cte_initial_energy(self.phi_ini, Gc, prob.ell, prob.h, A)
        self.phi = self.phi_ini.copy()
        self.H = self.psi_ini.copy()
        self.x = np.zeros((prob.s,) + prob.n)
        self.E = 0.0
        self.Sigma = 0.0
        self.T = 0.0
        self.tau = model.dissipation(self.phi, Gc, prob.ell, prob.h, A)
        self.tau0 = self.tau
        self.step = 0
        self.fractured = False
        self.curve = [dict(step=0, E=0.0, Sigma=0.0, T=0.0, D=self.tau,
                           Gamma=model.crack_surface(self.phi, prob.ell, prob.h, A), tau=self.tau)]


def fractured(prob, phi):
    broken = (phi >= prob.frac_threshold) | prob.mat.void
    return bool(np.all(np.any(broken, axis=prob.load_axis)))


class StepNotConverged(RuntimeError):
    pass


class StaggerNotConverged(StepNotConverged):
    pass


class ConstraintNotConverged(StepNotConverged):
    pass


def step(prob, st, dtau):
    """One dissipation-controlled step tau^{n+1} = tau^n + dtau (Eq. 16).

    At an unstable crack advance the staggered map can stall (its fixed
    point is approached no further; Sec. 4.1 has the paper relax its Newton
    steps for the same reason).  Dissipation control allows any subdivision
    of the increment, so an attempt that fails leaves the state unchanged
    and is replaced by two attempts of half its increment, recursively, at
    most max_halvings levels deep.  If the deepest one fails as well, the
    state returns to what it was when the step began and the failure is
    raised.  Returns the record of the last (sub)step.
    """
    saved = copy.deepcopy(st)
    try:
        return _step_split(prob, st, dtau, 0)
    except StepNotConverged:
        st.__dict__.update(saved.__dict__)
        raise


def _step_split(prob, st, dtau, depth):
    try:
        return _step_once(prob, st, dtau)
    except StepNotConverged:
        if depth >= prob.max_halvings:
            raise
        _step_split(prob, st, 0.5 * dtau, depth + 1)
        return _step_split(prob, st, 0.5 * dtau, depth + 1)


def _step_once(prob, st, dtau):
    """One step without subdivision.  The stagger map phi -> phi_new (one
    (M) then one (A)) is iterated to its fixed point; the iterates are
    combined by Anderson mixing of depth prob.anderson_depth (least squares
    on the last residual differences), which leaves the fixed point
    unchanged and only shortens the way there.  The attempt fails after
    max_stagger iterations, or once its error has not been halved for
    stall_window iterations (a stall).  The state is changed only once the
    stagger has converged.
    """
    tau = st.tau + dtau
    phi, E, x = st.phi.copy(), st.E, st.x.copy()
    n_cg = n_solves = 0
    err = math.inf
    hist_F, hist_G = [], []
    m = prob.anderson_depth
    ref, ref_it = math.inf, 0
    for it in range(1, prob.max_stagger + 1):
        x, ncg = mechanics(prob, phi, x)
        n_cg += ncg
        _, _, psi1, _ = unit_response(prob, phi, x)
        E_new, phi_new, ns = arclength(prob, psi1, st.psi_ini, st.H, tau, E)
        n_solves += ns
        dphi = math.sqrt(_dot(phi_new - phi, phi_new - phi)) / max(math.sqrt(_dot(phi_new, phi_new)), 1e-300)
        dE = abs(E_new - E) / max(abs(E_new), 1e-300)
        err = max(dphi, dE)
        E = E_new
        if err < 0.5 * ref:
            ref, ref_it = err, it
        if err < prob.tol:
            phi = phi_new
            break
        if prob.stall_window > 0 and it - ref_it >= prob.stall_window:
            raise StaggerNotConverged("stagger stalled (err=%g)" % err)
        if m > 0:
            hist_F.append((phi_new - phi).ravel())
            hist_G.append(phi_new.ravel())
            if len(hist_F) > m + 1:
                hist_F.pop(0)
                hist_G.pop(0)
        if m > 0 and len(hist_F) >= 2:
            dF = np.stack([hist_F[i + 1] - hist_F[i] for i in range(len(hist_F) - 1)], axis=1)
            dG = np.stack([hist_G[i + 1] - hist_G[i] for i in range(len(hist_G) - 1)], axis=1)
            A = dF.T @ dF
            gamma = np.linalg.solve(A + 1e-14 * np.trace(A) * np.eye(A.shape[0]), dF.T @ hist_F[-1])
            phi = (hist_G[-1] - dG @ gamma).reshape(prob.n)
        else:
            phi = phi_new
    else:
        raise StaggerNotConverged("stagger did not converge (err=%g)" % err)
    x, ncg = mechanics(prob, phi, x)
    n_cg += ncg
    _, sig1, psi1, Sigma1 = unit_response(prob, phi, x)
    H_new = history_field(prob, E, psi1, st.psi_ini, st.H)
    Sigma = E * Sigma1
    st.T += 0.5 * (Sigma + st.Sigma) * (E - st.E)
    st.phi, st.E, st.x, st.H, st.Sigma, st.tau = phi, E, x, H_new, Sigma, tau
    st.step += 1
    st.fractured = fractured(prob, phi)
    rec = dict(step=st.step, E=E, Sigma=Sigma, T=st.T,
               D=model.dissipation(phi, prob.mat.Gc, prob.ell, prob.h, prob.mat.A),
               Gamma=model.crack_surface(phi, prob.ell, prob.h, prob.mat.A), tau=tau,
               n_stagger=it, n_cg=n_cg, n_damage_solves=n_solves, fractured=st.fractured)
    rec["G_inst"] = instantaneous_G(prob, st.curve[-1], rec)
    st.curve.append(rec)
    return rec


def dissipated_by_curve(rec):
    """Energy per unit volume dissipated up to a point of the curve: the
    area under Sigma(E) minus the elastic energy still stored,
    T - 1/2 Sigma E (Eq. 33 at that point)."""
    return rec["T"] - 0.5 * rec["Sigma"] * rec["E"]


def instantaneous_G(prob, prev, rec):
    """Instantaneous energy release rate between two consecutive points of
    the curve (Sec. 4.2, Eq. 34): the change of the dissipated energy over
    the change of the crack surface Gamma (Eq. 4),
    G = V [(T - 1/2 Sigma E)^n - (T - 1/2 Sigma E)^(n-1)] / (Gamma^n - Gamma^(n-1)).
    Eq. 34 prints the difference of T alone; the text defines G as the
    variation of the dissipation, and T also carries the change of the
    stored elastic energy, so the dissipated part of the curve is used.
    None when Gamma did not grow."""
    dG = rec["Gamma"] - prev["Gamma"]
    if not dG > 0.0:
        return None
    return prob.V * (dissipated_by_curve(rec) - dissipated_by_curve(prev)) / dG


def effective_toughness(prob, st):
    """G_eff = V (T^f - 1/2 Sigma^f E^f) / A_g (Eq. 32-33)."""
    return prob.V * (st.T - 0.5 * st.Sigma * st.E) / prob.A_g


def run(prob, dtau, max_steps=10000, callback=None):
    st = State(prob)
    while not st.fractured and st.step < max_steps:
        rec = step(prob, st, dtau)
        if callback is not None:
            callback(rec)
    return st, (effective_toughness(prob, st) if st.fractured else None)
