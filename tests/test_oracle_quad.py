"""Pins of the oracle's multi-point triangle quadrature (no GPU): the rules integrate polynomials
of their degree exactly, the one-point rule is the centroid oracle, and the 3- and 6-point
energies are pinned by the scaling law, rigid motions, finite differences and convergence to the
exact double integral of two separated triangles."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M

DEGREE = {1: 1, 3: 2, 6: 4}


@pytest.mark.parametrize("rule", [1, 3, 6])
def test_rule_exactness(rule):
    # reference triangle (0,0), (1,0), (0,1): int x^a y^b = a! b! / (a + b + 2)!
    b, w = oracle.quad_rule(rule)
    assert w.sum() == pytest.approx(1.0, abs=1e-14) and np.allclose(b.sum(1), 1.0, atol=1e-15)
    x, y = b[:, 1], b[:, 2]
    for deg in range(DEGREE[rule] + 1):
        for a in range(deg + 1):
            exact = math.factorial(a) * math.factorial(deg - a) / math.factorial(deg + 2)
            assert 0.5 * (w * x ** a * y ** (deg - a)).sum() == pytest.approx(exact, rel=1e-13, abs=1e-15)
    # and not beyond: some monomial of the next degree is missed
    deg = DEGREE[rule] + 1
    miss = [abs(0.5 * (w * x ** a * y ** (deg - a)).sum()
                - math.factorial(a) * math.factorial(deg - a) / math.factorial(deg + 2)) for a in range(deg + 1)]
    assert max(miss) > 1e-6


def test_one_point_rule_is_the_centroid_oracle():
    X, F = M.icosphere(2)
    X = M.radial_jitter(X, 0.03, 4)
    E1, G1 = oracle.gradient_quad(X, F, 1)
    E, G = oracle.gradient(X, F)
    assert E1 == pytest.approx(E, rel=1e-13)
    assert np.abs(G1 - G).max() <= 1e-12 * np.abs(G).max()


@pytest.mark.parametrize("rule", [3, 6])
def test_scaling_and_rigid_motion(rule):
    X, F = M.icosphere(1)
    X = M.radial_jitter(X, 0.05, 2)
    E, G = oracle.gradient_quad(X, F, rule)
    E2, G2 = oracle.gradient_quad(3.0 * X, F, rule)
    assert E2 == pytest.approx(E / 9.0, rel=1e-12)
    assert np.abs(G2 - G / 27.0).max() <= 1e-11 * np.abs(G).max() / 27.0
    R = M.random_rotation(3)
    E3, G3 = oracle.gradient_quad(X @ R.T - 0.4, F, rule)
    assert E3 == pytest.approx(E, rel=1e-12)
    assert np.abs(G3 - G @ R.T).max() <= 1e-10 * np.abs(G).max()
    # zero net force and torque
    assert np.abs(G.sum(0)).max() <= 1e-12 * np.abs(G).sum()
    assert np.abs(np.cross(X, G).sum(0)).max() <= 1e-12 * np.abs(G).sum()


@pytest.mark.parametrize("rule", [3, 6])
def test_gradient_finite_differences(rule):
    X, F = M.icosphere(1)
    X = M.radial_jitter(X, 0.02, 8)
    E, G = oracle.gradient_quad(X, F, rule)
    h = 1e-4
    Gfd = np.zeros_like(X)
    for v in range(X.shape[0]):
        for d in range(3):
            def e(t):
                Xt = X.copy(); Xt[v, d] += t
                return oracle.gradient_quad(Xt, F, rule, want_grad=False)[0]
            Gfd[v, d] = (8 * (e(h) - e(-h)) - (e(2 * h) - e(-2 * h))) / (12 * h)
    assert np.abs(G - Gfd).max() / np.abs(G).max() < 1e-8


def subdivide(X, F, levels):
    for _ in range(levels):
        nV = X.shape[0]
        e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
        uniq, inv = np.unique(e[:, 0] * (nV + 1) + e[:, 1], return_inverse=True)
        Mid = 0.5 * (X[uniq // (nV + 1)] + X[uniq % (nV + 1)])
        m = inv.reshape(3, -1).T + nV
        i, j, k = F[:, 0], F[:, 1], F[:, 2]
        F = np.stack([np.stack([i, m[:, 0], m[:, 2]], 1), np.stack([m[:, 0], j, m[:, 1]], 1),
                      np.stack([m[:, 2], m[:, 1], k], 1), np.stack([m[:, 0], m[:, 1], m[:, 2]], 1)], 1).reshape(-1, 3)
        X = np.concatenate([X, Mid])
    return X, F.astype(np.int32)


def cross_energy(XS, FS, XT, FT, rule):
    """Energy of the pairs between the two separate surfaces (both orders)."""
    X = np.concatenate([XS, XT]); F = np.concatenate([FS, FT + XS.shape[0]]).astype(np.int32)
    e = lambda X_, F_: oracle.gradient_quad(X_, F_, rule, want_grad=False)[0]
    return e(X, F) - e(XS, FS) - e(XT, FT)


def test_convergence_to_the_double_integral():
    # two separated, tilted triangles; reference: the 6-point rule on 4^4 subtriangles of each
    S = np.array([[0, 0, 0], [1, 0, 0], [0.2, 0.9, 0.1]], float)
    T = np.array([[0.3, 0.1, 1.6], [1.2, 0.4, 1.9], [0.1, 1.0, 1.7]], float)
    F1 = np.array([[0, 1, 2]], np.int32)
    XS, FS = subdivide(S, F1, 4)
    XT, FT = subdivide(T, F1, 4)
    ref = cross_energy(XS, FS, XT, FT, 6)
    err = {r: abs(cross_energy(S, F1, T, F1, r) - ref) / ref for r in (1, 3, 6)}
    assert err[6] < err[3] < err[1] and err[6] < 1e-3 and err[1] > 1e-2
