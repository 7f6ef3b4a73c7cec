"""Spectral operators of the FFT solver (oracle; test infrastructure only).

Sec. 4.1: the equilibrium residual is written as the Fourier-Galerkin
convolution of the stress with a projection (Eq. 24 R1, Eq. 26), and the
gradient / divergence of the damage residual are evaluated in Fourier space
(Eq. 24 R2, Eq. 25 J2).

The DFT is numpy's unnormalised forward transform F[u](k) = sum_x u(x)
exp(-2 pi i k.x / N) with inverse 1/N sum_k ...  Grids are periodic with
voxel size h; index j of an axis of length N maps to the signed wavenumber
k in [-N/2, N/2).

Readings of the paper taken here:

* Projection.  Eq. 26 prints the projection for non-symmetric tensors; the
  unknowns are symmetric strains, so the symmetric projection onto
  compatible strains is used:  P(n):t = n(x)(t n) + (t n)(x)n - (n.t.n) n(x)n
  with n = xi/|xi|, and P = 0 at xi = 0.  It has the same null space
  (t n = 0, i.e. equilibrium), is idempotent and self-adjoint.
* Mechanical frequencies.  xi_j = 2 pi k_j / (N_j h).  On an axis of even
  length the Nyquist index k_j = -N_j/2 keeps xi_j = -pi/h only when every
  other index of that frequency is zero; otherwise that xi_j is set to 0.
  This keeps P(xi(-k)) = P(xi(k)) so real fields map to real fields.
* Damage derivatives.  The gradient uses the forward-difference symbols
  d_j = (exp(2 pi i k_j / N_j) - 1) / h and the divergence the negative
  adjoint, -conj(d_j).
"""
import numpy as np

from . import mandel


def signed_indices(N):
    """Signed wavenumbers of an axis of length N, in FFT storage order."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)


def mechanical_xi(n, h):
    """Frequency vectors xi[j, *n] (Sec. 4.1, Eq. 26) with the Nyquist rule."""
    d = len(n)
    ks = np.meshgrid(*[signed_indices(N) for N in n], indexing="ij")
    xi = np.zeros((d,) + tuple(n))
    for j in range(d):
        xi[j] = 2.0 * np.pi * ks[j] / (n[j] * h)
    for j in range(d):
        if n[j] % 2 == 0:
            nyq = ks[j] == -n[j] // 2
            others_zero = np.ones(tuple(n), dtype=bool)
            for i in range(d):
                if i != j:
                    others_zero &= ks[i] == 0
            xi[j][nyq & ~others_zero] = 0.0
    return xi


def projection_matrices(n, h):
    """Mandel matrices P[*n, s, s] of the compatible-strain projection (Eq. 26).

    Column b is P(n):t_b for the b-th Mandel basis tensor t_b, evaluated at
    every frequency; P = 0 where xi = 0.
    """
    d = len(n)
    s = mandel.nsym(d)
    xi = np.moveaxis(mechanical_xi(n, h), 0, -1)          # [*n, d]
    nrm = np.sqrt(np.sum(xi * xi, axis=-1, keepdims=True))
    nv = np.divide(xi, nrm, out=np.zeros_like(xi), where=nrm > 0)
    nn = np.einsum("...i,...j->...ij", nv, nv)
    P = np.zeros(tuple(n) + (s, s))
    basis = np.eye(s)
    for b in range(s):
        t = mandel.mandel_to_tensor(basis[b], d)                 # [d, d]
        tn = np.einsum("ij,...j->...i", t, nv)                   # t n
        ntn = np.einsum("...i,...i->...", nv, tn)                # n.t.n
        pt = (np.einsum("...i,...j->...ij", nv, tn) + np.einsum("...i,...j->...ij", tn, nv)
              - ntn[..., None, None] * nn)
        P[..., :, b] = mandel.tensor_to_mandel(pt, d)
    return P


def fft_fields(u):
    """Forward DFT over the spatial axes of a [c, *n] stack of fields."""
    return np.fft.fftn(u, axes=tuple(range(1, u.ndim)))


def ifft_fields(U):
    return np.fft.ifftn(U, axes=tuple(range(1, U.ndim)))


def green_apply(tau, P):
    """Eq. 24 R1 / Eq. 25 J1: F^-1{ P : F[tau] } for a [s, *n] Mandel field."""
    T = fft_fields(tau)
    out = np.einsum("...ab,b...->a...", P, T)
    res = ifft_fields(out)
    return res.real


def difference_symbols(n, h):
    """Forward-difference symbols d[j, *n] = (exp(2 pi i k_j / N_j) - 1) / h."""
    d = len(n)
    ks = np.meshgrid(*[np.arange(N) for N in n], indexing="ij")
    return np.stack([(np.exp(2j * np.pi * ks[j] / n[j]) - 1.0) / h for j in range(d)])


def gradient(phi, dsym):
    """Discrete gradient F^-1[d phi_hat] of a scalar field -> [d, *n]."""
    ph = np.fft.fftn(phi)
    return np.stack([np.fft.ifftn(dsym[j] * ph).real for j in range(dsym.shape[0])])


def divergence(v, dsym):
    """Discrete divergence F^-1[sum_j -conj(d_j) F[v_j]] of a [d, *n] field."""
    acc = np.zeros(v.shape[1:], dtype=complex)
    for j in range(v.shape[0]):
        acc += -np.conj(dsym[j]) * np.fft.fftn(v[j])
    return np.fft.ifftn(acc).real
