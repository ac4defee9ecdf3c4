"""Pins of the oracle's curved cubic (P3) elements (no GPU).

- The element map reproduces any cubic polynomial map exactly, with its derivatives: positions
  and Jacobians of curved elements are checked against a polynomial the test differentiates by
  hand, independent of the Lagrange basis.
- Straight elements (nodes at their lattice points) give the flat multi-point scheme: the same
  energy, and the flat gradient is the P3 gradient pulled back through the linear node map.
- The gradient matches central differences of the energy on a curved, jittered mesh, at corner,
  edge and centre nodes.
- Rigid motions leave the energy unchanged, scaling follows E(sX) = s^(4+q-p) E(X), and the
  gradient carries no net force or torque.
"""
import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M


def _cubic_map(seed):
    """Random cubic map (s, t) -> R^3 with its partial derivatives."""
    rng = np.random.default_rng(seed)
    terms = [(i, j) for i in range(4) for j in range(4 - i)]
    C = rng.normal(size=(len(terms), 3))

    def f(s, t):
        x = sum(C[k] * s ** i * t ** j for k, (i, j) in enumerate(terms))
        xs = sum(C[k] * i * s ** (i - 1) * t ** j for k, (i, j) in enumerate(terms) if i > 0)
        xt = sum(C[k] * j * s ** i * t ** (j - 1) for k, (i, j) in enumerate(terms) if j > 0)
        return x, xs, xt
    return f


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_map_reproduces_cubics(seed):
    f = _cubic_map(seed)
    # node k at reference point (s, t) = (l1, l2) of its lattice point
    P = np.array([f(l[1], l[2])[0] for l in M.P3_LATTICE])
    rng = np.random.default_rng(100 + seed)
    for _ in range(20):
        s, t = rng.uniform(0, 1, 2)
        if s + t > 1:
            s, t = 1 - s, 1 - t
        x, xs, xt = oracle.p3_map(P, s, t)
        x0, xs0, xt0 = f(s, t)
        scale = np.abs(P).max()
        assert np.abs(x - x0).max() <= 1e-13 * scale
        assert np.abs(xs - xs0).max() <= 1e-12 * scale
        assert np.abs(xt - xt0).max() <= 1e-12 * scale


def test_basis_is_nodal():
    # the basis interpolates: node k alone at 1 gives 1 at node k and 0 at the others
    for k in range(10):
        P = np.zeros((10, 3))
        P[k, 0] = 1.0
        for m, l in enumerate(M.P3_LATTICE):
            x, _, _ = oracle.p3_map(P, l[1], l[2])
            assert x[0] == pytest.approx(1.0 if m == k else 0.0, abs=1e-14)


def _node_map(X, F, X10, F10):
    """Matrix A with X10 = A X for straight elements (each node a fixed affine combination of
    its element's corners)."""
    A = np.zeros((X10.shape[0], X.shape[0]))
    for f in range(F.shape[0]):
        for k in range(10):
            A[F10[f, k], F[f]] = M.P3_LATTICE[k]
    return A


@pytest.mark.parametrize("rule", [1, 3, 6])
@pytest.mark.parametrize("qp", [(6.0, 12.0), (4.0, 8.0)])
def test_straight_elements_are_the_flat_scheme(rule, qp):
    q, p = qp
    X, F = M.icosphere(1)
    X = M.radial_jitter(X, 0.05, 3)
    X10, F10 = M.p3_lattice(X, F)
    A = _node_map(X, F, X10, F10)
    assert np.abs(A @ X - X10).max() < 1e-15
    E3, G3 = oracle.gradient_p3(X10, F10, rule, q, p)
    Ef, Gf = oracle.gradient_quad(X, F, rule, q, p)
    assert E3 == pytest.approx(Ef, rel=1e-12)
    assert np.abs(A.T @ G3 - Gf).max() <= 1e-11 * np.abs(Gf).max()


def _curved(seed=5, level=1, jitter=0.02):
    X10, F10 = M.p3_sphere(level, 2, 4, 0.05, seed)
    rng = np.random.default_rng(seed)
    return X10 + rng.normal(0.0, jitter, X10.shape) * 0.1, F10


@pytest.mark.parametrize("rule", [3, 6])
def test_gradient_matches_finite_differences(rule):
    X10, F10 = _curved()
    E, G = oracle.gradient_p3(X10, F10, rule)
    h = 1e-6
    # single coordinates of a corner, an edge node and a centre node of element 0
    for node in (F10[0, 0], F10[0, 4], F10[0, 9], F10[7, 6]):
        for d in range(3):
            Xp, Xm = X10.copy(), X10.copy()
            Xp[node, d] += h
            Xm[node, d] -= h
            fd = (oracle.gradient_p3(Xp, F10, rule, want_grad=False)[0]
                  - oracle.gradient_p3(Xm, F10, rule, want_grad=False)[0]) / (2 * h)
            assert fd == pytest.approx(G[node, d], rel=2e-6, abs=1e-7 * np.abs(G).max())
    # random directions through every node at once
    rng = np.random.default_rng(9)
    for _ in range(3):
        U = rng.normal(size=X10.shape)
        fd = (oracle.gradient_p3(X10 + h * U, F10, rule, want_grad=False)[0]
              - oracle.gradient_p3(X10 - h * U, F10, rule, want_grad=False)[0]) / (2 * h)
        assert fd == pytest.approx(float((G * U).sum()), rel=1e-6)


def test_rigid_motions_scaling_and_balance():
    X10, F10 = _curved(seed=7)
    q, p = 6.0, 12.0
    E, G = oracle.gradient_p3(X10, F10, 6, q, p)
    R = M.random_rotation(11)
    Er, _ = oracle.gradient_p3(X10 @ R.T + np.array([0.3, -1.2, 2.0]), F10, 6, q, p, want_grad=False)
    assert Er == pytest.approx(E, rel=1e-12)
    s = 1.7
    Es, _ = oracle.gradient_p3(s * X10, F10, 6, q, p, want_grad=False)
    assert Es == pytest.approx(s ** (4 + q - p) * E, rel=1e-12)
    gmax = np.abs(G).max()
    assert np.abs(G.sum(axis=0)).max() <= 1e-11 * gmax * G.shape[0]
    torque = np.cross(X10, G).sum(axis=0)
    assert np.abs(torque).max() <= 1e-11 * gmax * G.shape[0]


def test_invalid_inputs():
    X10, F10 = M.p3_sphere(1, coeff_std=0.0)
    bad = F10.copy()
    bad[0, 5] = X10.shape[0]
    with pytest.raises(oracle.OracleError):
        oracle.gradient_p3(X10, bad, 3)
    with pytest.raises(oracle.OracleError):
        oracle.gradient_p3(X10, F10, 4)
