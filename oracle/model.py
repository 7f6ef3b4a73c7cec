"""Material model, AT2 functionals, damage operator, crack-tip enrichment.

Oracle; test infrastructure only.  Arrays are indexed [x, y(, z)]: array
axis j is spatial direction j.  (The public input layout is the reverse,
x fastest in memory; ``solver.Problem`` transposes once on entry.)

Readings of the paper taken here:

* Degradation (Sec. 2.1).  The paper prints g = (1 - phi)^2 - k, which is
  negative at phi = 1; the residual stiffness is added:
  g = (1 - phi)^2 + k, g' = -2 (1 - phi) (Eq. 6).
* Void notch (Sec. 4.3).  A notch voxel has stiffness k * C of its phase,
  no elastic driving force (psi_0 = 0) and its phase's G_c.
* Discrete damage derivatives.  Forward differences with periodic wrap;
  the operator L(phi) = -div(G_c l A grad phi) of Eq. 10b / 17 is
  sum_jk D_j^T diag(G_c l A_jk) D_k with D the forward difference, A the
  voxel's cleavage tensor (Eq. 15) applied to the forward-difference
  gradient at the voxel (A = I when beta = 0).
* Cleavage tensor (Sec. 2.2, Eq. 15).  A = I + beta (I - n n) with n the
  phase's weak-plane normal (lattice axes) rotated by the voxel's angle
  about z; in 2D, n is its projection on the plane, normalised (A = (1 +
  beta) I when the normal is along z).
* Crack-tip enrichment (Eq. 35).  The smoothing solves
  phi_o + l^2 D^T D phi_o = phi_disc (the printed l in front of the
  Laplacian is taken as l^2 for consistent units).
* Initial energy (Eq. 37a, 38).  psi_ini = gamma_f'(phi_ini) / (2 (1 - phi_ini)),
  clamped at zero, which makes phi_ini the damage solution at zero load.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mandel, spectral


# --------------------------------------------------------------------------
# materials
# --------------------------------------------------------------------------

def phase_stiffness(phase, d, theta=0.0, R=None):
    """Mandel stiffness of one phase, rotated by R (Eq. 12-13); without R,
    about z by theta."""
    if phase["kind"] == "iso":
        C4 = mandel.isotropic_c4(phase["E"], phase["nu"])
    elif phase["kind"] == "cubic":
        C4 = mandel.cubic_c4(phase["C11"], phase["C12"], phase["C44"])
    else:
        raise ValueError("unknown phase kind")
    C4r = mandel.rotate_c4(C4, mandel.rotation_z(theta) if R is None else R)
    return mandel.c4_to_mandel(C4r, d), mandel.bulk_modulus_c4(C4r)


def cleavage_tensor(phase, d, theta=0.0, R=None):
    """A_f = I + beta (I - n n) of one phase (Eq. 15) with n the unit lattice
    normal rotated by R (without R, about z by theta); in 2D its in-plane
    block, which is what the projection of the rotated normal on the cross
    section gives (Sec. 5.3): a normal along z weakens every in-plane
    direction alike, A = (1 + beta) I."""
    beta = float(phase.get("beta", 0.0))
    I = np.eye(d)
    if beta == 0.0:
        return I
    n = np.asarray(phase.get("n", (0.0, 0.0, 1.0)), dtype=float)
    norm = np.linalg.norm(n)
    if norm == 0.0:
        return (1.0 + beta) * I
    Rm = mandel.rotation_z(theta) if R is None else R
    n = Rm @ (n / norm)
    A = np.eye(3) + beta * (np.eye(3) - np.outer(n, n))
    return A[:d, :d]


class MaterialField:
    """Per-voxel stiffness C[*n, s, s], bulk modulus K, G_c, void flag and,
    when some phase has beta != 0, the cleavage tensor A[*n, d, d] (else
    A is None: the isotropic functionals).  Orientations: theta[*n] (about
    z) or euler[*n, 3] (z-x-z Euler angles, Sec. 5.3)."""

    def __init__(self, n, phases, phase_id, theta=None, void=None, k=1e-6, euler=None):
        n = tuple(n)
        d = len(n)
        s = mandel.nsym(d)
        self.n, self.d, self.s, self.k = n, d, s, k
        self.C = np.zeros(n + (s, s))
        self.K = np.zeros(n)
        self.Gc = np.zeros(n)
        self.void = np.zeros(n, dtype=bool) if void is None else void.astype(bool)
        aniso = any(float(ph.get("beta", 0.0)) != 0.0 for ph in phases)
        self.A = np.zeros(n + (d, d)) if aniso else None
        cache = {}
        assert theta is None or euler is None
        for idx in np.ndindex(*n):
            p = int(phase_id[idx])
            if euler is not None:
                ang = tuple(float(v) for v in euler[idx])
            else:
                ang = (0.0 if theta is None else float(theta[idx]), 0.0, 0.0)
            R = mandel.rotation_euler(*ang)
            key = (p, ang)
            if key not in cache:
                cache[key] = phase_stiffness(phases[p], d, R=R)
            C, K = cache[key]
            scale = k if self.void[idx] else 1.0
            self.C[idx] = scale * C
            self.K[idx] = scale * K
            self.Gc[idx] = phases[p]["Gc"]
            if aniso:
                self.A[idx] = cleavage_tensor(phases[p], d, R=R)


def degradation(phi, k):
    """g(phi) = (1 - phi)^2 + k (Sec. 2.1, sign of k read as +)."""
    return (1.0 - phi) ** 2 + k


def stress_undegraded(eps, mat):
    """sigma_o = C : eps for a [s, *n] Mandel strain field (Eq. 2, 12)."""
    return np.einsum("...ab,b...->a...", mat.C, eps)


def stress(eps, phi, mat, split="none"):
    """Degraded stress (Eq. 10a / 16a integrand).

    split = "none": sigma = g(phi) C:eps (the paper's model, Eq. 2).
    split = "voldev": tension/compression split on the volumetric part,
      sigma = g (C:eps - K tr(eps) I + K <tr eps>_+ I) + K <tr eps>_- I,
      valid for isotropic and cubic stiffness where C:I = 3K I.
    """
    g = degradation(phi, mat.k)
    s0 = stress_undegraded(eps, mat)
    if split == "none":
        return g * s0
    tr = _trace(eps, mat.d)
    I = _identity(mat.d)
    pos = np.maximum(tr, 0.0)
    neg = np.minimum(tr, 0.0)
    vol_full = mat.K * tr
    out = np.empty_like(s0)
    for a in range(mat.s):
        out[a] = g * (s0[a] - I[a] * vol_full + I[a] * mat.K * pos) + I[a] * mat.K * neg
    return out


def energy_density(eps, mat, split="none"):
    """Undegraded elastic energy psi_o = 1/2 eps:C:eps (Eq. 2); 0 on voids.

    With split = "voldev" only the tensile part psi_o^+ drives damage.
    """
    s0 = stress_undegraded(eps, mat)
    psi = 0.5 * np.sum(eps * s0, axis=0)
    if split == "voldev":
        tr = _trace(eps, mat.d)
        psi = psi - 0.5 * mat.K * tr ** 2 + 0.5 * mat.K * np.maximum(tr, 0.0) ** 2
    return np.where(mat.void, 0.0, psi)


def _trace(eps, d):
    return eps[0] + eps[1] + (eps[2] if d == 3 else 0.0)


def _identity(d):
    return np.array([1.0, 1.0, 0.0]) if d == 2 else np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])


# --------------------------------------------------------------------------
# AT2 functionals (Eq. 3, 4) and the damage operator (Eq. 10b, 17, 24 R2)
# --------------------------------------------------------------------------

def forward_difference(phi, axis, h):
    """(phi(x + h e_j) - phi(x)) / h with periodic wrap."""
    return (np.roll(phi, -1, axis=axis) - phi) / h


def backward_difference_adjoint(v, axis, h):
    """D_j^T v = (v(x - h e_j) - v(x)) / h (adjoint of the forward difference)."""
    return (np.roll(v, 1, axis=axis) - v) / h


def _grad_A_grad(phi, h, A):
    """grad phi . A grad phi per voxel, forward-difference gradient."""
    d = phi.ndim
    g = [forward_difference(phi, j, h) for j in range(d)]
    if A is None:
        return sum(gj * gj for gj in g)
    return sum(A[..., j, k] * g[j] * g[k] for j in range(d) for k in range(d))


def dissipation(phi, Gc, ell, h, A=None):
    """D(phi) = int G_c (phi^2 / 2l + l/2 A : grad phi grad phi) (Eq. 3, 14)."""
    d = phi.ndim
    dens = phi ** 2 / (2.0 * ell) + 0.5 * ell * _grad_A_grad(phi, h, A)
    return float(np.sum(Gc * dens) * h ** d)


def crack_surface(phi, ell, h, A=None):
    """Gamma(phi) = int (phi^2 / 2l + l/2 A : grad phi grad phi) (Eq. 4)."""
    return dissipation(phi, np.ones_like(phi), ell, h, A)


def damage_operator(phi, Gc, ell, h, A=None):
    """L(phi) = -div(G_c l A grad phi) = sum_jk D_j^T (G_c l A_jk D_k phi) (Eq. 17)."""
    d = phi.ndim
    g = [forward_difference(phi, k, h) for k in range(d)]
    out = np.zeros_like(phi)
    for j in range(d):
        flux = g[j] if A is None else sum(A[..., j, k] * g[k] for k in range(d))
        out += backward_difference_adjoint(Gc * ell * flux, j, h)
    return out


def damage_operator_fft(phi, Gc, ell, dsym):
    """The same operator in the paper's Fourier form (Eq. 24 R2):
    -F^-1[xi . F[G_c l F^-1[xi phi_hat]]] with the difference symbols."""
    grad = spectral.gradient(phi, dsym)
    return -spectral.divergence(Gc * ell * grad, dsym)


def gamma_prime(phi, Gc, ell, h, A=None):
    """gamma_f'(phi) = G_c phi / l - div(G_c l A grad phi) (Eq. 17)."""
    return Gc * phi / ell + damage_operator(phi, Gc, ell, h, A)


def _difference_matrix_1d(N, h):
    idx = np.arange(N)
    S = sp.csr_matrix((np.ones(N), (idx, (idx + 1) % N)), shape=(N, N))
    return (S - sp.identity(N, format="csr")) / h


def difference_matrices(n, h):
    """Sparse forward differences D_j acting on C-order flattened [x, y, z] arrays."""
    mats = []
    for j in range(len(n)):
        M = sp.identity(1, format="csr")
        for i, N in enumerate(n):
            M = sp.kron(M, _difference_matrix_1d(N, h) if i == j else sp.identity(N), format="csr")
        mats.append(M)
    return mats


def gradient_matrix(coef, Dmats, A=None):
    """sum_jk D_j^T diag(coef A_jk) D_k (A = I when None)."""
    d = len(Dmats)
    M = None
    for j in range(d):
        for k in range(d):
            if A is None and j != k:
                continue
            c = coef if A is None else coef * A[..., j, k]
            term = Dmats[j].T @ sp.diags(np.ravel(c)) @ Dmats[k]
            M = term if M is None else M + term
    return M


def damage_matrix(H, Gc, ell, Dmats, A=None):
    """Matrix of the damage system (G_c/l + 2H) phi + L phi = 2H (Eq. 10b / 16b
    with H in place of psi_o, Eq. 11, 17)."""
    diag = (Gc / ell + 2.0 * H).ravel()
    return (sp.diags(diag) + gradient_matrix(Gc * ell, Dmats, A)).tocsc()


def factor_damage(H, Gc, ell, Dmats, A=None):
    """Sparse LU factors of the damage matrix; .solve(b) applies its inverse."""
    return spla.splu(damage_matrix(H, Gc, ell, Dmats, A))


def solve_damage(H, Gc, ell, Dmats, rhs=None, A=None):
    """phi solving (G_c/l + 2H) phi + L phi = 2H (or the given rhs), direct."""
    M = damage_matrix(H, Gc, ell, Dmats, A)
    b = (2.0 * H if rhs is None else rhs).ravel()
    return spla.spsolve(M, b).reshape(H.shape)


# --------------------------------------------------------------------------
# crack-tip enrichment (Sec. 4.3, Eq. 35, 37a, 38)
# --------------------------------------------------------------------------

def cte_initial_damage(phi_disc, ell, h, phi_M, A=None, Dmats=None):
    """phi_o + l^2 D^T A D phi_o = phi_disc; phi_ini = phi_M phi_o / max phi_o
    (Eq. 35; Eq. 36 with the cleavage tensor A, solved directly then)."""
    n = phi_disc.shape
    if not np.any(phi_disc > 0):
        return np.zeros(n)
    if A is None:
        dsym = spectral.difference_symbols(n, h)
        lap = np.sum(np.abs(dsym) ** 2, axis=0)
        phio = np.fft.ifftn(np.fft.fftn(phi_disc) / (1.0 + ell ** 2 * lap)).real
    else:
        M = sp.identity(int(np.prod(n))) + gradient_matrix(np.full(n, ell * ell), Dmats, A)
        phio = spla.spsolve(M.tocsc(), np.ravel(phi_disc).astype(float)).reshape(n)
    return phi_M * phio / np.max(phio)


def cte_initial_energy(phi_ini, Gc, ell, h, A=None):
    """psi_ini = max(0, gamma_f'(phi_ini) / (2 (1 - phi_ini))) (Eq. 37a / 37b, sign read)."""
    return np.maximum(gamma_prime(phi_ini, Gc, ell, h, A) / (2.0 * (1.0 - phi_ini)), 0.0)
