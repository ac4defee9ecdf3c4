"""Pins of the FP64 NumPy reference network against central finite differences (CPU)."""
import numpy as np

from oracle import mlp_ref


def test_reference_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = sum(int(np.prod(s)) for s in mlp_ref.SHAPES)
    assert n == 11472
    p = rng.normal(0, 0.3, n)
    X = rng.normal(size=(40, 32))
    T = np.concatenate([rng.normal(size=(40, 15)), rng.uniform(0.5, 1.5, (40, 1))], 1)
    g = mlp_ref.gradient(p, X, T)
    h = 1e-6
    for idx in rng.choice(n, 60, replace=False):
        e = np.zeros(n); e[idx] = h
        fd = (mlp_ref.loss(p + e, X, T) - mlp_ref.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])) + 1e-8, (idx, fd, g[idx])


def test_reference_loss_ignores_unused_rows_and_columns():
    rng = np.random.default_rng(1)
    n = sum(int(np.prod(s)) for s in mlp_ref.SHAPES)
    p = rng.normal(0, 0.3, n)
    X = rng.normal(size=(10, 32))
    T = np.concatenate([rng.normal(size=(10, 15)), np.ones((10, 1))], 1)
    L = mlp_ref.loss(p, X, T)
    T2 = T.copy(); T2[:, 7:15] = 99.0  # unused output columns
    assert mlp_ref.loss(p, X, T2) == L
    X3 = np.concatenate([X, rng.normal(size=(5, 32))]); T3 = np.concatenate([T, np.zeros((5, 16))])
    assert abs(mlp_ref.loss(p, X3, T3) - L) <= 1e-13 * L
