"""Mandel notation and stiffness tensors (oracle; test infrastructure only).

Symmetric second-order tensors are stored as Mandel vectors so that the
double contraction a:b equals the Euclidean dot product of the vectors:

  2D (plane strain, in-plane part)  [t_xx, t_yy, sqrt2 t_xy]                     s = 3
  3D                                [t_xx, t_yy, t_zz, sqrt2 t_yz, sqrt2 t_xz,
                                     sqrt2 t_xy]                                 s = 6

Fourth-order stiffness tensors are built as full 3x3x3x3 arrays (isotropic,
cubic) and rotated with the 81-term contraction of Eq. 13 (Sec. 2.2); the
Mandel matrix is read off the rotated full tensor.  Plane strain keeps the
in-plane block (Sec. 5: one-voxel-thick plates; the in-plane and anti-plane
parts decouple for isotropic phases and for cubic phases rotated about z).
"""
import numpy as np

SQ2 = np.sqrt(2.0)


def mandel_index_pairs(d):
    """Tensor index pairs (i, j) of each Mandel slot."""
    if d == 2:
        return [(0, 0), (1, 1), (0, 1)]
    if d == 3:
        return [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    raise ValueError("dimension must be 2 or 3")


def nsym(d):
    return 3 if d == 2 else 6


def _weights(d):
    return np.array([1.0 if i == j else SQ2 for (i, j) in mandel_index_pairs(d)])


def tensor_to_mandel(t, d):
    """[..., d, d] symmetric tensor -> [..., s] Mandel vector."""
    pairs = mandel_index_pairs(d)
    w = _weights(d)
    return np.stack([w[a] * t[..., i, j] for a, (i, j) in enumerate(pairs)], axis=-1)


def mandel_to_tensor(v, d):
    """[..., s] Mandel vector -> [..., d, d] symmetric tensor."""
    pairs = mandel_index_pairs(d)
    w = _weights(d)
    t = np.zeros(v.shape[:-1] + (d, d), dtype=v.dtype)
    for a, (i, j) in enumerate(pairs):
        t[..., i, j] = v[..., a] / w[a]
        t[..., j, i] = v[..., a] / w[a]
    return t


def c4_to_mandel(C4, d):
    """Full 3x3x3x3 stiffness -> s x s Mandel matrix of its d-dimensional block."""
    pairs = mandel_index_pairs(d)
    w = _weights(d)
    s = len(pairs)
    M = np.zeros((s, s))
    for a, (i, j) in enumerate(pairs):
        for b, (k, l) in enumerate(pairs):
            M[a, b] = w[a] * w[b] * C4[i, j, k, l]
    return M


def isotropic_c4(E, nu):
    """Isotropic stiffness C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    I = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))


def cubic_c4(C11, C12, C44):
    """Cubic stiffness in lattice axes: C_1111 = C11, C_1122 = C12, C_1212 = C44."""
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            if i == j:
                C[i, i, i, i] = C11
            else:
                C[i, i, j, j] = C12
                C[i, j, i, j] = C44
                C[i, j, j, i] = C44
    return C


def rotation_z(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rotation_x(angle):
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rotation_euler(phi1, Phi, phi2):
    """Lattice-to-sample rotation of the Euler angles (phi1, Phi, phi2) in the
    z-x-z convention: R = R_z(phi1) R_x(Phi) R_z(phi2) (Sec. 5.3 draws grain
    orientations as three Euler angles; (phi1, 0, 0) is the in-plane angle
    phi1)."""
    return rotation_z(phi1) @ rotation_x(Phi) @ rotation_z(phi2)


def rotate_c4(C4, R):
    """Eq. 13: C^r_ijkl = R_im R_jn R_kp R_lq C_mnpq."""
    return np.einsum("im,jn,kp,lq,mnpq->ijkl", R, R, R, R, C4)


def bulk_modulus_c4(C4):
    """K with C:I = 3K I (isotropic and cubic tensors); K = (C_iijj)/9."""
    return np.einsum("iijj->", C4) / 9.0


def zener_ratio(C11, C12, C44):
    """Eq. 40: z = 2 C_1212 / (C_1111 - C_1122)."""
    return 2.0 * C44 / (C11 - C12)
