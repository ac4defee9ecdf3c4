"""Seeded synthetic surface meshes (closed triangulated spheres and their deformations).

These generators produce the workloads on which the tangent-point energy is evaluated:
icospheres, radial jitter, real spherical-harmonic deformations, an invagination bump that
brings two sheets of the surface close together, and seeded rigid rotations.  They hold none
of the energy's arithmetic; both the HIP path and the CPU oracle consume their output.

All functions return ``(X, F)`` with ``X`` float64 [V, 3] vertex positions and ``F`` int32
[nF, 3] vertex indices, 0-based, consistently oriented (outward normals on the sphere).
Faces come in hierarchical subdivision order: the four children of a parent face are
consecutive, so nearby faces tend to have nearby indices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosphere", "radial_jitter", "real_sph_harm", "sh_deform", "sh_deform_amplitude",
    "bump", "random_rotation", "make_config", "CONFIGS", "ConfigMesh", "n_faces", "n_vertices",
    "P3_LATTICE", "p3_lattice", "p3_sphere",
]


def n_faces(level: int) -> int:
    return 20 * 4 ** level


def n_vertices(level: int) -> int:
    return 10 * 4 ** level + 2


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    X = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return X, F


def icosphere(level: int, radius: float = 1.0):
    """Unit icosphere refined ``level`` times by 1:4 midpoint subdivision.

    Vertex 0 is the icosahedron vertex (0, 1, t)/|.| at every level, and its antipode is vertex 3.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    X, F = _icosahedron()
    for _ in range(level):
        nV = X.shape[0]
        # unique undirected edges -> midpoint vertex ids
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        e_sorted = np.sort(e, axis=1)
        key = e_sorted[:, 0] * (nV + 1) + e_sorted[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        a = uniq // (nV + 1)
        b = uniq % (nV + 1)
        M = X[a] + X[b]
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        mid = inv.reshape(3, -1).T + nV  # [nF, 3]: ab, bc, ca
        ab, bc, ca = mid[:, 0], mid[:, 1], mid[:, 2]
        i, j, k = F[:, 0], F[:, 1], F[:, 2]
        C = np.stack([
            np.stack([i, ab, ca], 1), np.stack([ab, j, bc], 1),
            np.stack([ca, bc, k], 1), np.stack([ab, bc, ca], 1),
        ], axis=1).reshape(-1, 3)
        X = np.concatenate([X, M], axis=0)
        F = C
    return X * radius, F.astype(np.int32)


def radial_jitter(X: np.ndarray, std: float, seed: int) -> np.ndarray:
    """r_v <- r_v (1 + eps_v), eps_v ~ N(0, std^2) i.i.d. (std is a standard deviation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = rng.normal(0.0, std, size=X.shape[0])
    return X * (1.0 + eps)[:, None]


def _sph_angles(U: np.ndarray):
    z = np.clip(U[:, 2], -1.0, 1.0)
    phi = np.arctan2(U[:, 1], U[:, 0])
    return z, phi


def real_sph_harm(lmax: int, U: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonics Y_lm at unit vectors U [n,3].

    Returns [(lmax+1)^2, n], row index l*l + l + m for m = -l..l.  m > 0 uses cos(m phi),
    m < 0 uses sin(|m| phi); all rows are orthonormal on the unit sphere.
    Fully normalised associated Legendre functions by the standard three-term recurrence.
    """
    z, phi = _sph_angles(U)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    n = U.shape[0]
    out = np.empty(((lmax + 1) ** 2, n))
    pmm = np.full(n, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * pmm
        p_lm2 = None
        p_lm1 = pmm
        cm = np.cos(m * phi) * math.sqrt(2.0) if m > 0 else None
        sm = np.sin(m * phi) * math.sqrt(2.0) if m > 0 else None
        for l in range(m, lmax + 1):
            if l == m:
                p = pmm
            elif l == m + 1:
                p = math.sqrt(2.0 * m + 3.0) * z * pmm
            else:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                p = a * (z * p_lm1 - b * p_lm2)
            if l > m:
                p_lm2, p_lm1 = p_lm1, p
            if m == 0:
                out[l * l + l] = p
            else:
                out[l * l + l + m] = p * cm
                out[l * l + l - m] = p * sm
    return out


_SH_CHUNK = 32768  # vertices per evaluation of the basis for large meshes (bounds its memory)


def _sh_field(U: np.ndarray, lmin: int, lmax: int, a: np.ndarray) -> np.ndarray:
    """f(u) = sum_{l=lmin..lmax, m} a_lm Y_lm(u); meshes above 200,000 vertices are evaluated in
    chunks of vertices so that the (lmax+1)^2 x n basis never exists at once."""
    rows = np.arange(lmin * lmin, (lmax + 1) ** 2)
    if U.shape[0] <= 200_000:
        return a @ real_sph_harm(lmax, U)[rows]
    return np.concatenate([a @ real_sph_harm(lmax, U[i:i + _SH_CHUNK])[rows]
                           for i in range(0, U.shape[0], _SH_CHUNK)])


def sh_deform(X: np.ndarray, lmin: int, lmax: int, coeff_std: float, seed: int):
    """r(u) = 1 + sum_{l=lmin..lmax, m} a_lm Y_lm(u),  a_lm ~ N(0, coeff_std^2)  on the unit directions of X."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = X / np.linalg.norm(X, axis=1, keepdims=True)
    a = rng.normal(0.0, coeff_std, size=(lmax + 1) ** 2 - lmin * lmin)
    r = 1.0 + _sh_field(U, lmin, lmax, a)
    if r.min() <= 0.2:
        raise ValueError("deformation not star-shaped enough (min r <= 0.2)")
    return U * r[:, None], a


def sh_deform_amplitude(X: np.ndarray, lmin: int, lmax: int, amplitude: float, seed: int):
    """White N(0,1) coefficients for l = lmin..lmax, rescaled so that max_v |r_v - 1| = amplitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U = X / np.linalg.norm(X, axis=1, keepdims=True)
    a = rng.normal(0.0, 1.0, size=(lmax + 1) ** 2 - lmin * lmin)
    f = _sh_field(U, lmin, lmax, a)
    a = a * (amplitude / np.abs(f).max())
    r = 1.0 + f * (amplitude / np.abs(f).max())
    if r.min() <= 0.2:
        raise ValueError("deformation not star-shaped enough (min r <= 0.2)")
    return U * r[:, None], a


def _min_dist(A: np.ndarray, B: np.ndarray, upper: float = np.inf) -> float:
    """Smallest distance between the point sets A and B; inf when it exceeds `upper`."""
    from scipy.spatial import cKDTree
    if A.shape[0] == 0 or B.shape[0] == 0:
        return float("inf")
    d, _ = cKDTree(B).query(A, k=1, distance_upper_bound=upper)
    return float(d.min())


def bump(X: np.ndarray, axis_vertex: int = 0, width: float = 0.3, gap: float = 0.02,
         depth: float | None = None, iters: int = 60):
    """Push a cap inward along -a (a = unit direction of ``axis_vertex``) by D exp(-g^2 / (2 width^2)),
    g = angle to a.  If ``depth`` is None, D is found by bisection so that the smallest distance
    between displaced-cap vertices (displacement > D/2) and undisplaced vertices (displacement
    < 1e-3 D) equals ``gap``.  Returns (X_new, D, realised_gap)."""
    U = X / np.linalg.norm(X, axis=1, keepdims=True)
    a = U[axis_vertex]
    gam = np.arccos(np.clip(U @ a, -1.0, 1.0))
    prof = np.exp(-gam ** 2 / (2.0 * width ** 2))

    def apply(D):
        return X - (D * prof)[:, None] * a[None, :]

    cap = np.flatnonzero(prof > 0.5)
    sheet = np.flatnonzero(prof < 1e-3)
    if depth is not None:
        Y = apply(depth)
        return Y, depth, _min_dist(Y[cap], Y[sheet])
    # The bisection only compares distances with `gap`, and reports the final one (~ gap).  The
    # displacement is along a, so distances perpendicular to a do not depend on D: a pair closer
    # than 2 gap is closer than 2 gap laterally.  Keeping only the sheet vertices within 2 gap of
    # some cap vertex laterally, and searching only up to 2 gap, leaves every comparison and the
    # reported gap exactly as over the whole sheet.
    bound = 2.0 * gap
    if cap.size and sheet.size:
        from scipy.spatial import cKDTree
        lat = X - (X @ a)[:, None] * a[None, :]
        d_lat, _ = cKDTree(lat[cap]).query(lat[sheet], k=1, distance_upper_bound=bound)
        sheet = sheet[np.isfinite(d_lat)]

    def gap_of(D):
        Y = apply(D)
        return _min_dist(Y[cap], Y[sheet], bound)

    lo, hi = 0.0, float(np.linalg.norm(X[axis_vertex]) + np.max(np.linalg.norm(X, axis=1)))
    # gap_of is decreasing in D until contact; bisect on gap_of(D) - gap
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        g = gap_of(mid)
        if g > gap:
            lo = mid
        else:
            hi = mid
    D = lo
    return apply(D), D, gap_of(D)


def random_rotation(seed: int) -> np.ndarray:
    """Uniform random rotation (QR of a Gaussian matrix with sign fix, det +1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.normal(size=(3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


@dataclass
class ConfigMesh:
    name: str
    X: np.ndarray
    F: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nF(self):
        return int(self.F.shape[0])

    @property
    def V(self):
        return int(self.X.shape[0])


def _c1(seed):
    X, F = icosphere(3)
    X = radial_jitter(X, 0.01, seed)
    return ConfigMesh("L3-jitter", X, F, {"level": 3, "jitter_std": 0.01, "seed": seed})


def _c2(seed):
    X, F = icosphere(5)
    X, a = sh_deform(X, 2, 8, 0.05, seed)
    return ConfigMesh("L5-sh8", X, F, {"level": 5, "sh_l": [2, 8], "coeff_std": 0.05, "seed": seed})


def _c3(seed, level=6, gap=0.02):
    X, F = icosphere(level)
    X, D, g = bump(X, 0, 0.3, gap)
    R = random_rotation(seed)
    X = X @ R.T
    return ConfigMesh(f"L{level}-bump", X, F,
                      {"level": level, "bump_width": 0.3, "gap_target": gap, "depth": D,
                       "gap": g, "seed": seed})


def _c4(seed, level=7):
    X, F = icosphere(level)
    X, a = sh_deform_amplitude(X, 2, 16, 0.15, seed)
    return ConfigMesh(f"L{level}-sh16", X, F,
                      {"level": level, "sh_l": [2, 16], "amplitude": 0.15, "seed": seed})


def _c5(seed, level=8):
    X, F = icosphere(level)
    X, a = sh_deform_amplitude(X, 2, 32, 0.2, seed)
    X, D, g = bump(X, 0, 0.3, 0.01)
    return ConfigMesh(f"L{level}-sh32-bump", X, F,
                      {"level": level, "sh_l": [2, 32], "amplitude": 0.2, "bump_width": 0.3,
                       "gap_target": 0.01, "depth": D, "gap": g, "seed": seed})


CONFIGS = {"C1": _c1, "C2": _c2, "C3": _c3, "C4": _c4, "C5": _c5}


# ---- curved cubic (P3) elements -----------------------------------------------------------------
# An element has 10 nodes at the barycentric lattice points of its flat parent (v0, v1, v2):
#   0, 1, 2: the corners; 3, 4: (2/3, 1/3, 0), (1/3, 2/3, 0); 5, 6: (0, 2/3, 1/3), (0, 1/3, 2/3);
#   7, 8: (1/3, 0, 2/3), (2/3, 0, 1/3); 9: (1/3, 1/3, 1/3).
# Neighbouring elements share their corner and edge nodes.

P3_LATTICE = np.array([[3, 0, 0], [0, 3, 0], [0, 0, 3],
                       [2, 1, 0], [1, 2, 0], [0, 2, 1], [0, 1, 2], [1, 0, 2], [2, 0, 1],
                       [1, 1, 1]], dtype=np.float64) / 3.0


def p3_lattice(X: np.ndarray, F: np.ndarray):
    """(X10, F10): the flat mesh (X, F) as straight cubic elements.  The first V nodes are the
    vertices of X (same indices), then two nodes per undirected edge, then one per face; every
    node sits at its lattice point, so the cubic map of each element is the flat triangle."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    V, nF = X.shape[0], F.shape[0]
    # directed face edges (i -> j) for the three sides 0-1, 1-2, 2-0
    I = F[:, [0, 1, 2]].reshape(-1)
    J = F[:, [1, 2, 0]].reshape(-1)
    lo, hi = np.minimum(I, J), np.maximum(I, J)
    key = lo * V + hi
    uk, inv = np.unique(key, return_inverse=True)
    ne = uk.shape[0]
    ulo, uhi = uk // V, uk % V
    # global edge nodes: V + 2 e (2/3 at lo), V + 2 e + 1 (2/3 at hi)
    near_lo = V + 2 * inv
    near_hi = near_lo + 1
    first = np.where(I == lo, near_lo, near_hi)    # the node 2/3 of the way at i
    second = np.where(I == lo, near_hi, near_lo)   # the node 2/3 of the way at j
    first, second = first.reshape(nF, 3), second.reshape(nF, 3)
    F10 = np.empty((nF, 10), dtype=np.int32)
    F10[:, 0:3] = F
    F10[:, 3], F10[:, 4] = first[:, 0], second[:, 0]
    F10[:, 5], F10[:, 6] = first[:, 1], second[:, 1]
    F10[:, 7], F10[:, 8] = first[:, 2], second[:, 2]
    F10[:, 9] = V + 2 * ne + np.arange(nF)
    X10 = np.empty((V + 2 * ne + nF, 3))
    X10[:V] = X
    X10[V:V + 2 * ne:2] = (2.0 * X[ulo] + X[uhi]) / 3.0
    X10[V + 1:V + 2 * ne:2] = (X[ulo] + 2.0 * X[uhi]) / 3.0
    X10[V + 2 * ne:] = X[F].mean(axis=1)
    return X10, F10


def p3_sphere(level: int, lmin: int = 2, lmax: int = 8, coeff_std: float = 0.05, seed: int = 0):
    """Curved cubic elements on the deformed sphere r(u) = 1 + sum a_lm Y_lm(u): the lattice nodes
    of the level-`level` icosphere are moved radially onto that surface (the corners land where
    ``sh_deform`` puts the vertices of the flat mesh with the same seed).  coeff_std = 0: the
    unit sphere."""
    X, F = icosphere(level)
    X10, F10 = p3_lattice(X, F)
    if coeff_std == 0.0:
        return X10 / np.linalg.norm(X10, axis=1, keepdims=True), F10
    X10, _ = sh_deform(X10, lmin, lmax, coeff_std, seed)
    return X10, F10


def make_config(name: str, seed: int = 0, **kw) -> ConfigMesh:
    """Workload presets.

    C1: level-3 icosphere (1,280 faces), radial jitter std 0.01.
    C2: level-5 (20,480 faces), SH l=2..8 with a_lm ~ N(0, 0.05^2).
    C3: level-6 (81,920 faces), inward bump of width 0.3 calibrated to a 0.02 gap, seeded rotation.
    C4: level-7 (327,680 faces), SH l=2..16 rescaled to max|r-1| = 0.15.
    C5: level-8 (1,310,720 faces), SH l=2..32 at max|r-1| = 0.2 plus a bump at gap 0.01.
    """
    return CONFIGS[name](seed, **kw)


def confinement_config(level: int = 5, conf_level: int = 5, radius: float = 1.1, flatten: float = 0.02,
                       seed: int = 0) -> tuple:
    """Sphere inside a spherical confinement (the paper's Sec. 4.2 setting): the unit icosphere of
    `level`, slightly flattened on one side (an inward Gaussian dent of depth `flatten` and width 0.3
    at vertex 0), and the concentric icosphere of `conf_level` scaled to `radius`, both turned by
    the same seeded rotation.  Returns (X, F, Y, FY)."""
    X, F = icosphere(level)
    X, _, _ = bump(X, 0, 0.3, depth=flatten)
    Y, FY = icosphere(conf_level)
    R = random_rotation(seed)
    return X @ R.T, F, (radius * Y) @ R.T, FY
