"""Pins of the FP64 NumPy reference network against central finite differences (CPU)."""
import numpy as np

from oracle import mlp_ref


import pytest


@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_reference_backprop_matches_finite_differences(lam):
    rng = np.random.default_rng(0)
    n = sum(int(np.prod(s)) for s in mlp_ref.SHAPES)
    assert n == 11472
    p = rng.normal(0, 0.3, n)
    X = rng.normal(size=(40, 32))
    T = np.concatenate([rng.normal(size=(40, 15)), rng.uniform(0.5, 1.5, (40, 1))], 1)
    g = mlp_ref.gradient(p, X, T, lam=lam, tile=16)
    h = 1e-6
    for idx in rng.choice(n, 60, replace=False):
        e = np.zeros(n); e[idx] = h
        fd = (mlp_ref.loss(p + e, X, T, lam, 16) - mlp_ref.loss(p - e, X, T, lam, 16)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])) + 1e-8, (idx, fd, g[idx])


def test_reference_difference_term():
    """The difference term sees only the row-to-row variation of the error inside a tile: it is
    unchanged when every target of a tile moves by the same amount (which changes the plain
    term), vanishes for a one-row tile, and does not couple rows of different tiles."""
    rng = np.random.default_rng(3)
    n = sum(int(np.prod(s)) for s in mlp_ref.SHAPES)
    p = rng.normal(0, 0.3, n)
    X = rng.normal(size=(12, 32))
    T = np.concatenate([rng.normal(size=(12, 15)), rng.uniform(0.5, 1.5, (12, 1))], 1)
    # the difference term itself: (loss with lam = 1) - (loss with lam = 0), times 7 sum w
    diff = lambda T_, tile: 7 * (mlp_ref.loss(p, X, T_, 1.0, tile) - mlp_ref.loss(p, X, T_, 0.0, tile))
    T2 = T.copy(); T2[4:8, :7] += rng.normal(size=7)  # rows 4..7 = tile 1 of tile size 4
    assert diff(T2, 4) * T2[:, 15].sum() == pytest.approx(diff(T, 4) * T[:, 15].sum(), rel=1e-12)
    assert mlp_ref.loss(p, X, T2) != mlp_ref.loss(p, X, T)
    assert diff(T, 1) == 0.0
    T3 = T.copy(); T3[4, :7] += 1.0  # a change in row 4 alters pairs (4,5) only with tile 4 ...
    d3 = diff(T3, 4) * T3[:, 15].sum() - diff(T, 4) * T[:, 15].sum()
    Y, _ = mlp_ref.forward(p, X)
    dd = (Y - T)[:, :7]
    w = T[:, 15]
    before = w[4] * w[5] * ((dd[5] - dd[4]) ** 2).sum()
    after = w[4] * w[5] * ((dd[5] - dd[4] + 1.0) ** 2).sum()
    assert d3 == pytest.approx(after - before, rel=1e-9)  # ... not (3,4): rows 3 and 4 are in different tiles


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
