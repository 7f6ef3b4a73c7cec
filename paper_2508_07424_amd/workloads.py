"""Seeded synthetic RVE workloads (microstructure geometry and load cases).

This module only draws geometry (which voxel belongs to which phase, where
the notch and its tips are) and lists the material constants and load of a
workload.  It holds none of the solver's arithmetic, so the test oracle and
the GPU library can both consume its output.

All arrays use the public layout: shape (n_y, n_x) in 2D or (n_z, n_y, n_x)
in 3D, C order, so x is the fastest index in memory.  Voxel centres sit at
(i + 1/2) h.  Distances are periodic.

The paper ships no RVE files (its composites, laminates and polycrystals are
described only in prose, Sec. 5), so the generators follow its prose:
random sequential adsorption of circular fibres (Sec. 5.2.2), periodic
Voronoi grains with in-plane orientations (Sec. 5.3), orthogonal laminates
(Sec. 5.1.2), and a one-voxel-thick notch row with crack-tip enrichment
points at its two ends (Sec. 4.3).
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    """One RVE toughness problem in the public layout."""
    n: tuple                      # (n_x, n_y[, n_z])
    h: float
    ell: float
    phases: List[dict]            # {"kind": "iso", E, nu, Gc} or {"kind": "cubic", C11, C12, C44, Gc}
    phase_id: np.ndarray          # uint16, shape reversed(n)
    f: np.ndarray                 # Mandel load direction (s,)
    dtau: float
    theta: Optional[np.ndarray] = None     # per-voxel in-plane angle (rad) or None
    void: Optional[np.ndarray] = None      # uint8 notch mask
    phi_disc: Optional[np.ndarray] = None  # uint8 enrichment points
    phi_M: float = 0.8
    k: float = 1e-6
    meta: dict = field(default_factory=dict)
    euler: Optional[np.ndarray] = None     # per-voxel z-x-z Euler angles, shape reversed(n) + (3,)

    @property
    def dim(self):
        return len(self.n)

    @property
    def shape(self):
        return tuple(reversed(self.n))


def _centres(n, h):
    """Voxel-centre coordinates, one array per axis, in public layout."""
    axes = [(np.arange(N) + 0.5) * h for N in n]
    grids = np.meshgrid(*axes, indexing="ij")          # [x, y, z] indexing
    return [np.ascontiguousarray(g.T) for g in grids]  # public layout


def _periodic_delta(a, b, L):
    d = np.abs(a - b) % L
    return np.minimum(d, L - d)


def rsa_disks(n, h, rng, radius_sampler, *, count=None, vf=None, min_gap=1.0,
              forbidden=None, max_tries=200000):
    """Random sequential adsorption of non-overlapping periodic disks/spheres.

    Disks are added until ``count`` are placed or the voxel volume fraction
    reaches ``vf``.  ``forbidden(centre, r)`` may veto a candidate.  Returns
    (list of (centre, r), mask of inclusion voxels in public layout).
    """
    d = len(n)
    L = np.array(n, dtype=float) * h
    coords = _centres(n, h)
    mask = np.zeros(tuple(reversed(n)), dtype=bool)
    placed = []
    tries = 0
    while True:
        if count is not None and len(placed) >= count:
            break
        if vf is not None and mask.mean() >= vf:
            break
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA could not place more inclusions")
        r = float(radius_sampler(rng))
        c = rng.uniform(0.0, 1.0, size=d) * L
        ok = True
        for (c2, r2) in placed:
            dist = math.sqrt(sum(_periodic_delta(c[j], c2[j], L[j]) ** 2 for j in range(d)))
            if dist < r + r2 + min_gap:
                ok = False
                break
        if ok and forbidden is not None and forbidden(c, r):
            ok = False
        if not ok:
            continue
        dist2 = sum(_periodic_delta(coords[j], c[j], L[j]) ** 2 for j in range(d))
        mask |= dist2 <= r * r
        placed.append((c, r))
    return placed, mask


def notch_2d(n, h, row, x0, x1):
    """A notch row y = row, x in [x0, x1): void mask and tip points."""
    nx, ny = n
    void = np.zeros((ny, nx), dtype=np.uint8)
    void[row, x0:x1] = 1
    tips = np.zeros((ny, nx), dtype=np.uint8)
    tips[row, x0] = 1
    tips[row, x1 - 1] = 1
    return void, tips


def notch_3d_square(n, h, zrow, x0, x1, y0, y1):
    """A square notch in plane z = zrow: void mask and its boundary voxels
    (the crack front, used as enrichment points)."""
    nx, ny, nz = n
    void = np.zeros((nz, ny, nx), dtype=np.uint8)
    void[zrow, y0:y1, x0:x1] = 1
    tips = np.zeros_like(void)
    tips[zrow, y0:y1, x0] = 1
    tips[zrow, y0:y1, x1 - 1] = 1
    tips[zrow, y0, x0:x1] = 1
    tips[zrow, y1 - 1, x0:x1] = 1
    return void, tips


def load_yy(dim):
    """f = e_y (x) e_y in Mandel form (Eq. 39)."""
    f = np.zeros(3 if dim == 2 else 6)
    f[1] = 1.0
    return f


def load_zz():
    f = np.zeros(6)
    f[2] = 1.0
    return f


def iso(E, nu, Gc):
    return {"kind": "iso", "E": float(E), "nu": float(nu), "Gc": float(Gc)}


def cubic(C11, C12, C44, Gc):
    return {"kind": "cubic", "C11": float(C11), "C12": float(C12), "C44": float(C44), "Gc": float(Gc)}


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def composite_2d_small(seed=1):
    """64 x 64 two-phase composite, 10 disks of radius 6 (plain FP64 case).

    Matrix E=1, nu=0.3, Gc=1; inclusions E=5, nu=0.25, Gc=2; l = 1.5 h;
    16-voxel notch along x at mid-height with enrichment at both tips;
    uniaxial y load; dtau = 0.01 Gc L_x.
    """
    n = (64, 64)
    h = 1.0
    r = 6.0
    row = 32
    yc = (row + 0.5) * h

    def forbidden(c, rad):
        return _periodic_delta(c[1], yc, n[1] * h) < rad + 2.0

    rng = np.random.default_rng(seed)
    _, mask = rsa_disks(n, h, rng, lambda g: r, count=10, forbidden=forbidden)
    void, tips = notch_2d(n, h, row, 24, 40)
    pid = mask.astype(np.uint16)
    return Workload(n=n, h=h, ell=1.5, phases=[iso(1, 0.3, 1), iso(5, 0.25, 2)],
                    phase_id=pid, f=load_yy(2), dtau=0.01 * 1.0 * n[0] * h,
                    void=void, phi_disc=tips, phi_M=0.8, k=1e-6,
                    meta={"name": "composite_2d_64", "vf": float(mask.mean()), "seed": seed})


def composite_2d(n=256, seed=1, E_ratio=5.0, Gc_ratio=2.0, vf=0.3, ell=2.0, crack=40,
                 rmin=5.0, rmax=9.0):
    """n x n fibre composite: disks with r ~ U[rmin, rmax] up to volume
    fraction vf, elastic and toughness contrasts, a crack-voxel notch."""
    nn = (n, n)
    h = 1.0
    row = n // 2
    yc = (row + 0.5) * h

    def forbidden(c, rad):
        return _periodic_delta(c[1], yc, n * h) < rad + 2.0 and \
            _periodic_delta(c[0], (n // 2) * h, n * h) < crack / 2 + rad + 2.0

    rng = np.random.default_rng(seed)
    placed, mask = rsa_disks(nn, h, rng, lambda g: g.uniform(rmin, rmax), vf=vf,
                             forbidden=forbidden)
    x0 = n // 2 - crack // 2
    void, tips = notch_2d(nn, h, row, x0, x0 + crack)
    return Workload(n=nn, h=h, ell=ell,
                    phases=[iso(1, 0.3, 1), iso(E_ratio, 0.25, Gc_ratio)],
                    phase_id=mask.astype(np.uint16), f=load_yy(2), dtau=0.01 * n * h,
                    void=void, phi_disc=tips, phi_M=0.8, k=1e-6,
                    meta={"name": "composite_2d_%d" % n, "fibres": len(placed),
                          "vf": float(mask.mean()), "seed": seed})


def two_phase_plate_2d(seed=21, n=(12, 10), dtau=0.12):
    """Small two-phase plate: each voxel stiff (E = 4, Gc = 2) with
    probability 0.4, else soft (E = 1, Gc = 1); a notch of voxels x = 3..6
    in row 5; l = 1.5, tension along y.  Small enough for Newton systems
    solved without a preconditioner."""
    rng = np.random.default_rng(seed)
    pid = (rng.random((n[1], n[0])) < 0.4).astype(np.uint16)
    void, tips = notch_2d(n, 1.0, 5, 3, 7)
    pid[void.astype(bool)] = 0
    return Workload(n=n, h=1.0, ell=1.5, phases=[iso(1, 0.3, 1), iso(4, 0.25, 2)], phase_id=pid,
                    f=load_yy(2), dtau=dtau, void=void, phi_disc=tips)


def homogeneous_2d(nx=32, ny=32, ell=1.5, crack=8, E=1.0, nu=0.3, Gc=1.0, phi_M=0.8,
                   dtau_frac=0.01):
    """Homogeneous plate with a centred notch (the 'broken in two' check)."""
    n = (nx, ny)
    h = 1.0
    row = ny // 2
    x0 = nx // 2 - crack // 2
    void, tips = notch_2d(n, h, row, x0, x0 + crack)
    return Workload(n=n, h=h, ell=ell, phases=[iso(E, nu, Gc)],
                    phase_id=np.zeros((ny, nx), dtype=np.uint16), f=load_yy(2),
                    dtau=dtau_frac * Gc * nx * h, void=void, phi_disc=tips, phi_M=phi_M,
                    k=1e-6, meta={"name": "homogeneous_2d_%dx%d" % (nx, ny)})


def laminate_2d(nx=64, ny=32, widths=(0.5, 0.5), Gcs=(1.0, 3.0), Es=(1.0, 1.0), nus=(0.3, 0.3),
                ell=1.5, crack_frac=0.1):
    """Orthogonal laminate: layers normal to x (the crack, along x, crosses
    them), notch of crack_frac L_x starting at x = 0 at mid-height."""
    n = (nx, ny)
    h = 1.0
    pid = np.zeros((ny, nx), dtype=np.uint16)
    edges = np.round(np.cumsum((0.0,) + tuple(widths)) * nx).astype(int)
    for p in range(len(widths)):
        pid[:, edges[p]:edges[p + 1]] = p
    row = ny // 2
    a = max(2, int(round(crack_frac * nx)))
    void, tips = notch_2d(n, h, row, 0, a)
    tips[row, 0] = 0          # the notch starts at the periodic boundary: one tip
    phases = [iso(Es[p], nus[p], Gcs[p]) for p in range(len(widths))]
    return Workload(n=n, h=h, ell=ell, phases=phases, phase_id=pid, f=load_yy(2),
                    dtau=0.01 * min(Gcs) * nx * h, void=void, phi_disc=tips, phi_M=0.8,
                    k=1e-6, meta={"name": "laminate_2d", "edges": edges.tolist()})


def inclusion_2d(n=24, radius=4.0, centre=(18.0, 12.0), E_ratio=3.0, Gc_ratio=2.0, ell=1.5,
                 crack=6):
    """n x n matrix (E = 1, nu = 0.3, Gc = 1) with one disk inclusion
    (E_ratio, nu = 0.25, Gc_ratio) at `centre` (voxel units) and a centred
    notch row of `crack` voxels at mid-height: a small case whose crack
    meets, grazes or misses the inclusion depending on where it starts."""
    nn = (n, n)
    h = 1.0
    X, Y = _centres(nn, h)
    d2 = _periodic_delta(X, centre[0] * h, n * h) ** 2 + _periodic_delta(Y, centre[1] * h, n * h) ** 2
    pid = (d2 <= (radius * h) ** 2).astype(np.uint16)
    row = n // 2
    x0 = n // 2 - crack // 2
    void, tips = notch_2d(nn, h, row, x0, x0 + crack)
    pid[void.astype(bool)] = 0
    return Workload(n=nn, h=h, ell=ell, phases=[iso(1.0, 0.3, 1.0), iso(E_ratio, 0.25, Gc_ratio)],
                    phase_id=pid, f=load_yy(2), dtau=0.01 * n * h, void=void, phi_disc=tips,
                    phi_M=0.8, k=1e-6, meta={"name": "inclusion_2d_%d" % n})


def _load_axis(w):
    """Index (0 x, 1 y, 2 z) of the largest normal component of the load."""
    d = len(w.n)
    return int(np.argmax(np.abs(np.asarray(w.f, dtype=float)[:d])))


def crack_position_samples(w, count):
    """The same RVE with the initial crack at `count` positions along the
    load axis (Sec. 3: the toughness estimate is the minimum over crack
    positions).  The RVE is periodic, so the microstructure (phase ids and
    orientations) is shifted cyclically by k L / count voxels along the load
    axis while the notch and its enrichment points stay where they are;
    notch voxels keep the phase they have in the unshifted RVE.  Returns
    [(shift, Workload)]."""
    a = _load_axis(w)
    d = len(w.n)
    axis = d - 1 - a                      # array axis of the load direction
    L = int(w.n[a])
    out = []
    for k in range(count):
        sh = int(round(k * L / count))
        pid = np.roll(w.phase_id, sh, axis=axis)
        th = None if w.theta is None else np.roll(w.theta, sh, axis=axis)
        if w.void is not None:
            pid = pid.copy()
            pid[w.void.astype(bool)] = w.phase_id[w.void.astype(bool)]
        meta = dict(w.meta)
        meta["crack_shift"] = sh
        out.append((sh, Workload(n=w.n, h=w.h, ell=w.ell, phases=w.phases, phase_id=pid, f=w.f,
                                 dtau=w.dtau, theta=th, void=w.void, phi_disc=w.phi_disc,
                                 phi_M=w.phi_M, k=w.k, meta=meta)))
    return out


def _voronoi_ids(X, Y, seeds, L):
    """Index of the nearest seed (periodic distance) of every voxel centre;
    ties go to the lower index."""
    try:
        from scipy.spatial import cKDTree
    except ImportError:
        cKDTree = None
    if cKDTree is not None and len(seeds) > 8:
        tree = cKDTree(np.mod(seeds, L), boxsize=L)
        pts = np.stack([np.mod(X.ravel(), L), np.mod(Y.ravel(), L)], axis=1)
        d, idx = tree.query(pts, k=2)
        # resolve exact ties like the brute-force scan (lowest index)
        tie = d[:, 0] == d[:, 1]
        best = np.where(tie, np.minimum(idx[:, 0], idx[:, 1]), idx[:, 0])
        return best.reshape(X.shape).astype(np.uint16)
    best = np.full(X.shape, np.inf)
    gid = np.zeros(X.shape, dtype=np.uint16)
    for g in range(len(seeds)):
        d2 = _periodic_delta(X, seeds[g, 0], L) ** 2 + _periodic_delta(Y, seeds[g, 1], L) ** 2
        closer = d2 < best
        best[closer] = d2[closer]
        gid[closer] = g
    return gid


def _laguerre_ids(X, Y, seeds, weights, L):
    """Index of the seed of least power distance |x - s|^2 - w (periodic) of
    every voxel centre: a weighted (Laguerre) Voronoi tessellation; ties go
    to the lower index."""
    best = np.full(X.shape, np.inf)
    gid = np.zeros(X.shape, dtype=np.uint16)
    for g in range(len(seeds)):
        d2 = (_periodic_delta(X, seeds[g, 0], L) ** 2 + _periodic_delta(Y, seeds[g, 1], L) ** 2
              - weights[g])
        closer = d2 < best
        best[closer] = d2[closer]
        gid[closer] = g
    return gid


def polycrystal_2d(n=512, grains=200, seed=1000, zener=2.0, a_cleave=1.0, ell=2.0,
                   crack_frac=0.1, beta=0.0, size_sigma=0.0):
    """Periodic Voronoi polycrystal with uniform in-plane orientations.

    Cubic C11 = 1, C12 = 0.5, C44 = z/4 (so 2 C44 / (C11 - C12) = z);
    per-grain Gc = 1 + a cos^2(4 theta).  Each grain is its own phase.
    beta > 0 gives every grain a cleavage plane (Sec. 5.3): the cubic [100]
    plane, weak-plane normal (1, 0, 0) in lattice axes, rotated with the
    grain.  size_sigma > 0 draws the grains as a weighted (Laguerre)
    tessellation whose seed radii are log-normal with that standard
    deviation of log r (Sec. 5.3 uses a weighted Voronoi with log-normal
    grain sizes); 0 gives the plain Voronoi tessellation.
    """
    nn = (n, n)
    h = 1.0
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, n * h, size=(grains, 2))
    theta_g = rng.uniform(0.0, 2.0 * np.pi, size=grains)
    X, Y = _centres(nn, h)
    if size_sigma > 0.0:
        r_mean = n * h / math.sqrt(math.pi * grains)
        radii = r_mean * np.exp(size_sigma * rng.standard_normal(grains) - 0.5 * size_sigma ** 2)
        gid = _laguerre_ids(X, Y, seeds, radii ** 2, n * h)
    else:
        gid = _voronoi_ids(X, Y, seeds, n * h)
    C44 = zener / 4.0
    phases = [cubic(1.0, 0.5, C44, 1.0 + a_cleave * math.cos(4.0 * t) ** 2) for t in theta_g]
    if beta != 0.0:
        phases = [dict(p, beta=float(beta), n=(1.0, 0.0, 0.0)) for p in phases]
    theta = theta_g[gid]
    row = n // 2
    a = max(2, int(round(crack_frac * n)))
    x0 = n // 2 - a // 2
    void, tips = notch_2d(nn, h, row, x0, x0 + a)
    return Workload(n=nn, h=h, ell=ell, phases=phases, phase_id=gid, f=load_yy(2),
                    dtau=0.01 * n * h, theta=theta, void=void, phi_disc=tips, phi_M=0.8,
                    k=1e-6, meta={"name": "polycrystal_2d_%d" % n, "grains": grains,
                                  "seed": seed, "zener": zener, "a": a_cleave, "beta": beta,
                                  "size_sigma": size_sigma})


def polycrystal_plate(n=64, layers=2, grains=30, seed=2000, zener=2.0, beta=1.0, ell=2.0,
                      crack_frac=0.1, size_sigma=0.0):
    """Polycrystal plate of Sec. 5.3: grains with orientations drawn in three
    dimensions (z-x-z Euler angles, uniform on the rotations: a1, a3 ~
    U[0, 2 pi), cos a2 ~ U[-1, 1]), cubic C11 = 1, C12 = 0.5, C44 = z/4,
    Gc = 1, cleavage on the cubic [100] plane with weight beta (on the
    cross section, the in-plane block of the rotated cleavage tensor: the
    projection of the rotated normal).  The paper's one-voxel plate is
    represented by `layers` identical layers along z (periodic, so the
    solution does not vary along z); the tessellation, notch (0.1 L_x at
    mid-height, through the thickness) and load e_y (x) e_y are those of
    polycrystal_2d.  dtau = 0.01 Gc L_x L_z."""
    h = 1.0
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, n * h, size=(grains, 2))
    a1 = rng.uniform(0.0, 2.0 * np.pi, size=grains)
    a2 = np.arccos(rng.uniform(-1.0, 1.0, size=grains))
    a3 = rng.uniform(0.0, 2.0 * np.pi, size=grains)
    X, Y = _centres((n, n), h)
    if size_sigma > 0.0:
        r_mean = n * h / math.sqrt(math.pi * grains)
        radii = r_mean * np.exp(size_sigma * rng.standard_normal(grains) - 0.5 * size_sigma ** 2)
        gid2 = _laguerre_ids(X, Y, seeds, radii ** 2, n * h)
    else:
        gid2 = _voronoi_ids(X, Y, seeds, n * h)
    phases = [dict(cubic(1.0, 0.5, zener / 4.0, 1.0), beta=float(beta), n=(1.0, 0.0, 0.0))
              for _ in range(grains)]
    euler2 = np.stack([a1[gid2], a2[gid2], a3[gid2]], axis=-1)
    a = max(2, int(round(crack_frac * n)))
    x0 = n // 2 - a // 2
    void2, tips2 = notch_2d((n, n), h, n // 2, x0, x0 + a)
    nn = (n, n, layers)
    rep = lambda arr: np.ascontiguousarray(np.broadcast_to(arr, (layers,) + arr.shape))
    f = np.zeros(6)
    f[1] = 1.0
    return Workload(n=nn, h=h, ell=ell, phases=phases, phase_id=rep(gid2), f=f,
                    dtau=0.01 * n * h * layers * h, void=rep(void2), phi_disc=rep(tips2), phi_M=0.8,
                    k=1e-6, euler=rep(euler2),
                    meta={"name": "polycrystal_plate_%d" % n, "grains": grains, "seed": seed,
                          "zener": zener, "beta": beta, "layers": layers})


def composite_3d(n=128, seed=1, spheres=40, vf=0.2, E_ratio=5.0, Gc_ratio=3.0, ell=2.0):
    """n^3 sphere composite; square notch L/2 x L/2 in the z mid-plane; z load."""
    nn = (n, n, n)
    h = 1.0
    r = (vf * n ** 3 / spheres * 3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    zc = (n // 2 + 0.5) * h

    def forbidden(c, rad):
        return _periodic_delta(c[2], zc, n * h) < rad + 2.0

    rng = np.random.default_rng(seed)
    _, mask = rsa_disks(nn, h, rng, lambda g: r, count=spheres, forbidden=forbidden)
    q = n // 4
    void, tips = notch_3d_square(nn, h, n // 2, q, q + n // 2, q, q + n // 2)
    return Workload(n=nn, h=h, ell=ell, phases=[iso(1, 0.3, 1), iso(E_ratio, 0.3, Gc_ratio)],
                    phase_id=mask.astype(np.uint16), f=load_zz(), dtau=0.01 * n * n * h * h,
                    void=void, phi_disc=tips, phi_M=0.8, k=1e-6,
                    meta={"name": "composite_3d_%d" % n, "r": r, "vf": float(mask.mean())})


def smooth_sizes(lo, hi):
    """Grid sizes in [lo, hi] whose prime factors are 2, 3, 5, 7, even."""
    out = []
    for n in range(lo, hi + 1):
        if n % 2:
            continue
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def serving_stream(count, seed=1, sizes_2d=(32, 48, 64, 96, 128), sizes_3d=(16, 24, 32),
                   frac_3d=0.25, rate=1.0, dtau_frac=0.02):
    """Requests of a serving run: list of (arrival seconds, Workload).

    Per request, from a seeded generator: the dimension (3D with probability
    frac_3d), the side log-uniform over the given 7-smooth sizes (a few
    sizes, so that requests of one size can share a batched pool),
    the microstructure (fibre/sphere composite or Voronoi polycrystal with
    probability 1/2 each; polycrystals in 2D only), elastic contrast
    U[1, 10] and toughness contrast U[1, 4].  Arrivals are a Poisson process
    of the given rate (requests per second).  dtau = dtau_frac Gc L (larger
    than the paper's 0.01 so that a request needs tens of steps).
    """
    rng = np.random.default_rng(seed)
    s2, s3 = sorted(sizes_2d), sorted(sizes_3d)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        three = rng.random() < frac_3d
        sizes = s3 if three else s2
        lw = np.log(sizes)
        pick = np.exp(rng.uniform(lw[0], lw[-1]))
        n = min(sizes, key=lambda v: abs(np.log(v) - np.log(pick)))
        e_c = float(rng.uniform(1.0, 10.0))
        g_c = float(rng.uniform(1.0, 4.0))
        s = int(rng.integers(1, 2 ** 31 - 1))
        if three:
            vol = n ** 3
            spheres = max(1, int(round(0.15 * vol / (4.0 / 3.0 * math.pi * (n / 6.0) ** 3))))
            w = composite_3d(n=n, seed=s, spheres=spheres, vf=0.15, E_ratio=e_c, Gc_ratio=g_c)
            w.dtau = dtau_frac * n * n
        elif rng.random() < 0.5:
            vf = float(rng.uniform(0.1, 0.3))
            w = composite_2d(n=n, seed=s, E_ratio=e_c, Gc_ratio=g_c, vf=vf, ell=2.0,
                             crack=max(2, n // 6), rmin=max(2.0, n / 40.0), rmax=max(3.0, n / 24.0))
            w.dtau = dtau_frac * n
        else:
            grains = max(4, int(round((n / 40.0) ** 2 * 4)))
            w = polycrystal_2d(n=n, grains=grains, seed=s, zener=float(rng.uniform(1.0, 4.0)),
                               a_cleave=float(rng.uniform(0.0, 3.0)), ell=2.0)
            w.dtau = dtau_frac * n
        w.meta.update({"request": i, "contrast_E": e_c, "contrast_Gc": g_c})
        out.append((t, w))
    return out
