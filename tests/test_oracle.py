"""Pins of the FP64 CPU oracle against what the definition and mathematics fix (no GPU).

The oracle evaluates the one-point centroid quadrature of the paper's tangent-point energy
(Sec. 2.2.2, eq. (TP)) over ordered face pairs sharing no vertex, and its exact vertex gradient.
Each test below checks it against something other than itself: closed forms, exact identities
(homogeneity, rigid-motion invariance), brute-force counts and central finite differences.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def two_triangles(s, h):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0],
                  [s, 0, h], [1 + s, 0, h], [s, 1, h]], dtype=np.float64)
    F = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    return X, F


def load_two_triangles():
    rows = []
    with open(os.path.join(GOLD, "two_triangles.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                s, h, q, p, E = line.split()
                rows.append((float(s), float(h), float(q), float(p), float(E)))
    return rows


@pytest.mark.parametrize("row", load_two_triangles())
def test_two_triangle_closed_form(row):
    s, h, q, p, E = row
    X, F = two_triangles(s, h)
    assert oracle.energy(X, F, q, p) == pytest.approx(E, rel=1e-13)
    # flipping either triangle's winding does not change |n.d|
    assert oracle.energy(X, F[:, ::-1].copy(), q, p) == pytest.approx(E, rel=1e-13)


def test_two_triangle_vertical_gradient():
    for h in (1.0, 0.5, 2.0):
        X, F = two_triangles(0.0, h)
        E, G = oracle.gradient(X, F)
        # translating the top triangle up by dh: dE/dh = -3 h^-7 for (q,p) = (6,12)
        assert G[3:, 2].sum() == pytest.approx(-3.0 * h ** -7, rel=1e-12)
        assert G[:3, 2].sum() == pytest.approx(3.0 * h ** -7, rel=1e-12)


def test_scale_is_linear():
    X, F = two_triangles(0.3, 0.9)
    E1 = oracle.energy(X, F)
    assert oracle.energy(X, F, scale=1e-4 / 6) == pytest.approx(E1 * 1e-4 / 6, rel=1e-14)


def test_adjacent_faces_are_excluded():
    # two triangles sharing exactly one vertex, or an edge, contribute nothing
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0.5], [0, -1, 0.3]], dtype=np.float64)
    F_vertex = np.array([[0, 1, 2], [0, 3, 4]], dtype=np.int32)
    assert oracle.energy(X, F_vertex) == 0.0
    F_edge = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    assert oracle.energy(X, F_edge) == 0.0
    E, G = oracle.gradient(X, F_edge)
    assert E == 0.0 and np.all(G == 0.0)


def test_pair_counts_brute_force():
    # ordered pairs of faces sharing no vertex, counted independently in Python
    for level in (1, 2):
        X, F = M.icosphere(level)
        sets = [set(f) for f in F.tolist()]
        n = sum(1 for a in sets for b in sets if not (a & b))
        assert oracle.pair_count(F) == n
    for level in (1, 2, 3, 4):
        X, F = M.icosphere(level)
        nF = F.shape[0]
        assert oracle.pair_count(F) == nF * nF - 13 * nF + 60


def test_flat_mesh_is_zero():
    # planar triangulated grid: n.d = 0 for every pair
    n = 6
    xs, ys = np.meshgrid(np.arange(n + 1.0), np.arange(n + 1.0), indexing="ij")
    X = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], 1) * 0.37
    idx = lambda i, j: i * (n + 1) + j
    F = []
    for i in range(n):
        for j in range(n):
            F.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)])
            F.append([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)])
    F = np.array(F, dtype=np.int32)
    R = M.random_rotation(3)
    X = X @ R.T + np.array([0.3, -1.0, 2.0])
    E, G = oracle.gradient(X, F)
    assert abs(E) < 1e-25
    assert np.abs(G).max() < 1e-12


def test_sphere_limit_convergence():
    """On a sphere of radius R the tangent-point radius is R everywhere (paper Sec. 2.2.2), so the
    continuum energy with (q,p) = (6,12) is (2R)^-6 (4 pi R^2)^2 = pi^2 / (4 R^2).  The centroid
    quadrature on refined icospheres must converge to it monotonically at second order."""
    errs = []
    for level in (1, 2, 3, 4):
        X, F = M.icosphere(level)
        errs.append(abs(oracle.energy(X, F) - np.pi ** 2 / 4) / (np.pi ** 2 / 4))
    for a, b in zip(errs, errs[1:]):
        assert b < a and a / b > 3.0
    assert errs[-1] < 2e-3
    # radius 2: same relative error, E scaled by 1/4
    X, F = M.icosphere(3)
    assert oracle.energy(2 * X, F) == pytest.approx(oracle.energy(X, F) / 4, rel=1e-13)


@pytest.mark.parametrize("q", [2.0, 4.0, 8.0])
def test_sphere_limit_other_exponents(q):
    """With p = 2q the kernel on a sphere of radius R is the constant (2R)^-q (the tangent-point
    radius is R everywhere), so the continuum energy of the unit sphere is (4 pi)^2 / 2^q.  The
    centroid quadrature must converge to it at second order."""
    ref = (4 * np.pi) ** 2 / 2 ** q
    errs = []
    for level in (1, 2, 3, 4):
        X, F = M.icosphere(level)
        errs.append(abs(oracle.energy(X, F, q, 2 * q) - ref) / ref)
    for a, b in zip(errs, errs[1:]):
        assert b < a and a / b > 3.0
    assert errs[-1] < 5e-3


@pytest.mark.parametrize("qp", [(6.0, 12.0), (4.0, 10.0), (8.0, 14.0)])
def test_scaling_law_and_euler(qp):
    q, p = qp
    X, F = M.icosphere(2)
    X = M.radial_jitter(X, 0.05, 11)
    E, G = oracle.gradient(X, F, q, p)
    for s in (0.5, 2.0, 3.7):
        assert oracle.energy(s * X, F, q, p) == pytest.approx(s ** (4 + q - p) * E, rel=1e-12)
    # Euler's identity for a function homogeneous of degree 4+q-p
    assert (X * G).sum() == pytest.approx((4 + q - p) * E, rel=1e-11)


def test_rigid_motion():
    X, F = M.icosphere(2)
    X = M.radial_jitter(X, 0.05, 5)
    E, G = oracle.gradient(X, F)
    scale = np.abs(G).max()
    assert np.abs(G.sum(0)).max() < 1e-12 * scale * X.shape[0]
    assert np.abs(np.cross(X, G).sum(0)).max() < 1e-12 * scale * X.shape[0]
    R = M.random_rotation(7)
    b = np.array([1.5, -0.25, 3.0])
    E2, G2 = oracle.gradient(X @ R.T + b, F)
    assert E2 == pytest.approx(E, rel=1e-12)
    assert np.abs(G2 - G @ R.T).max() < 1e-10 * scale


def test_orientation_and_permutation():
    X, F = M.icosphere(2)
    X = M.radial_jitter(X, 0.05, 9)
    E, G = oracle.gradient(X, F)
    rng = np.random.default_rng(1)
    F2 = F.copy()
    flip = rng.random(F.shape[0]) < 0.5
    F2[flip] = F2[flip][:, ::-1]
    E2, G2 = oracle.gradient(X, F2)
    assert E2 == pytest.approx(E, rel=1e-13)
    assert np.abs(G2 - G).max() < 1e-12 * np.abs(G).max()
    # relabel vertices and faces
    pv = rng.permutation(X.shape[0])
    inv = np.empty_like(pv)
    inv[pv] = np.arange(pv.size)
    X3 = X[pv]
    F3 = inv[F][rng.permutation(F.shape[0])].astype(np.int32)
    E3, G3 = oracle.gradient(X3, F3)
    assert E3 == pytest.approx(E, rel=1e-12)
    assert np.abs(G3 - G[pv]).max() < 1e-11 * np.abs(G).max()


def _fd_gradient(X, F, h, **kw):
    G = np.zeros_like(X)
    for v in range(X.shape[0]):
        for d in range(3):
            Xp = X.copy(); Xp[v, d] += h
            Xm = X.copy(); Xm[v, d] -= h
            Xp2 = X.copy(); Xp2[v, d] += 2 * h
            Xm2 = X.copy(); Xm2[v, d] -= 2 * h
            # fourth-order central difference
            G[v, d] = (8 * (oracle.energy(Xp, F, **kw) - oracle.energy(Xm, F, **kw))
                       - (oracle.energy(Xp2, F, **kw) - oracle.energy(Xm2, F, **kw))) / (12 * h)
    return G


def _patch(X, F, center, nfaces):
    """Open patch: the nfaces faces whose centroids are closest to `center`, reindexed."""
    c = X[F].mean(1)
    sel = np.argsort(np.linalg.norm(c - center, axis=1), kind="stable")[:nfaces]
    Fs = F[np.sort(sel)]
    used, inv = np.unique(Fs, return_inverse=True)
    return X[used].copy(), inv.reshape(Fs.shape).astype(np.int32)


def fd_meshes():
    X1, F1 = M.icosphere(1)
    yield "jittered-L1", M.radial_jitter(X1, 0.01, 0), F1
    X2, F2 = M.icosphere(2)
    Xb, _, _ = M.bump(X2, 0, 0.3, 0.15)
    yield "bumped-L2", Xb, F2
    X3, F3 = M.icosphere(3)
    Xb3, _, _ = M.bump(X3, 0, 0.3, 0.05)
    # both sheets across the gap, near the axis
    axis = Xb3[3] / np.linalg.norm(Xb3[3])
    Xp, Fp = _patch(Xb3, F3, axis * 0.97, 180)
    yield "gap-patch-L3", Xp, Fp


@pytest.mark.parametrize("name,X,F", list(fd_meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_gradient_finite_differences(name, X, F):
    E, G = oracle.gradient(X, F)
    assert E > 0
    h = 1e-4 * np.abs(X).max()
    Gfd = _fd_gradient(X, F, h)
    err = np.abs(G - Gfd).max() / np.abs(G).max()
    assert err < 1e-8, (name, err)


@pytest.mark.parametrize("qp", [(2.0, 4.0), (4.0, 8.0), (8.0, 10.0)])
def test_gradient_finite_differences_other_exponents(qp):
    """The exact path also runs other exponents; their oracle gradient is pinned the same way."""
    q, p = qp
    X, F = M.icosphere(1)
    X = M.radial_jitter(X, 0.03, 4)
    E, G = oracle.gradient(X, F, q, p)
    assert E > 0
    h = 1e-4 * np.abs(X).max()
    Gfd = _fd_gradient(X, F, h, q=q, p=p)
    err = np.abs(G - Gfd).max() / np.abs(G).max()
    assert err < 1e-8, (qp, err)


def test_gradient_at_matches_full():
    X, F = M.icosphere(3)
    X = M.radial_jitter(X, 0.01, 2)
    E, G = oracle.gradient(X, F)
    verts = np.array([0, 3, 17, 200, 641], dtype=np.int32)
    Gs = oracle.gradient_at(X, F, verts)
    assert np.abs(Gs - G[verts]).max() < 1e-12 * np.abs(G).max()


def test_energy_rows_partition():
    X, F = M.icosphere(3)
    X = M.radial_jitter(X, 0.01, 4)
    E = oracle.energy(X, F)
    parts = [oracle.energy_rows(X, F, a, b) for a, b in [(0, 100), (100, 777), (777, 1280)]]
    assert sum(parts) == pytest.approx(E, rel=1e-13)


def test_error_paths():
    X, F = two_triangles(0.5, 0.5)
    with pytest.raises(oracle.OracleError) as e:
        oracle.energy(X, np.array([[0, 1, 7], [3, 4, 5]], dtype=np.int32))
    assert e.value.code == -1
    Xd = X.copy(); Xd[2] = Xd[1]  # zero-area face
    with pytest.raises(oracle.OracleError) as e:
        oracle.energy(Xd, F)
    assert e.value.code == -2
    Xn = X.copy(); Xn[0, 0] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.energy(Xn, F)
    assert e.value.code == -3
    # coincident centroids of two faces that share no vertex: the energy is infinite
    Xc = np.concatenate([X[:3], X[:3] @ np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1.0]])], 0)
    with pytest.raises(oracle.OracleError) as e:
        oracle.energy(Xc, F)
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError):
        oracle.energy(X, F, q=6.0, p=5.0)


def test_row_ranges_add_up_to_the_whole():
    """The row-range form (the CPU baseline's bounded sample) splits the energy and gradient exactly
    along rows: the pieces add up to the full evaluation."""
    c = M.make_config("C1")
    E, G = oracle.gradient(c.X, c.F)
    parts = [oracle.gradient_rows(c.X, c.F, a, b) for a, b in ((0, 1), (1, 700), (700, 1280))]
    assert abs(sum(p[0] for p in parts) - E) <= 1e-13 * abs(E)
    assert np.abs(sum(p[1] for p in parts) - G).max() <= 1e-13 * np.abs(G).max()
    assert abs(oracle.energy_rows(c.X, c.F, 1, 700) - parts[1][0]) <= 1e-13 * abs(E)
