"""Shared helpers for the tests: build the oracle problem of a workload."""
import numpy as np

from oracle import solver


def oracle_problem(w, **kw):
    return solver.Problem(w.n, w.h, w.ell, w.phases, w.phase_id, w.f, theta=w.theta,
                          void=w.void, phi_disc=w.phi_disc, phi_M=w.phi_M, k=w.k,
                          euler=getattr(w, "euler", None), **kw)


def to_oracle(a, d):
    """Public layout (x fastest, optional leading component axis) -> [.., x, y, z]."""
    if a.ndim == d:
        return np.ascontiguousarray(a.T)
    return np.ascontiguousarray(a.transpose((0,) + tuple(range(a.ndim - 1, 0, -1))))


def relmax(a, b):
    """Element-wise deviation: max |a - b| over max |b|."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    den = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))
