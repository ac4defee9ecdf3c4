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


def test_bf16_rounding():
    """Round to nearest, ties to even, on the 7 stored mantissa bits of BF16."""
    one = 1.0
    assert mlp_ref.bf16(one) == 1.0
    assert mlp_ref.bf16(1 + 2.0 ** -8) == 1.0                   # tie -> even mantissa (0)
    assert mlp_ref.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6     # tie -> even mantissa (2)
    assert mlp_ref.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert mlp_ref.bf16(-3.0) == -3.0 and mlp_ref.bf16(0.0) == 0.0
    x = np.random.default_rng(0).normal(size=10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    r = mlp_ref.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))
    assert np.array_equal(mlp_ref.bf16(r), r)
    assert np.all(np.sign(r) == np.sign(x))


def test_low_precision_mode_reduces_to_the_exact_network():
    """With the rounding steps replaced by the identity the kernel-rounding mode is the FP64 network
    (so the two modes differ only where the kernels round), and with them it stays close to it."""
    rng = np.random.default_rng(4)
    n = sum(int(np.prod(s)) for s in mlp_ref.SHAPES)
    p = rng.normal(0, 0.2, n)
    X = rng.normal(size=(64, 32))
    T = np.concatenate([rng.normal(size=(64, 15)), rng.uniform(0.5, 1.5, (64, 1))], 1)
    ident = lambda a: np.asarray(a, dtype=np.float64)
    Y0, _ = mlp_ref.forward(p, X)
    Y1, _ = mlp_ref.forward(p, X, low=True, rnd=ident, store=ident)
    assert np.abs(Y1 - Y0).max() <= 1e-13 * np.abs(Y0).max()
    g0 = mlp_ref.gradient(p, X, T, lam=0.3, tile=16)
    g1 = mlp_ref.gradient(p, X, T, lam=0.3, tile=16, low=True, rnd=ident, store=ident)
    assert np.abs(g1 - g0).max() <= 1e-12 * np.abs(g0).max()
    Yb, _ = mlp_ref.forward(p, X, low=True)
    gb = mlp_ref.gradient(p, X, T, lam=0.3, tile=16, low=True)
    assert 0 < np.abs(Yb - Y0).max() <= 5e-2 * np.abs(Y0).max()
    assert float(gb @ g0 / (np.linalg.norm(gb) * np.linalg.norm(g0))) > 0.999


def test_adam_first_step_is_a_signed_step():
    """With zero moments, the bias-corrected first Adam step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    p1, m1, v1 = mlp_ref.adam(p, np.zeros(100), np.zeros(100), g, 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # a second step with the same gradient: m = 0.19 g, v = 0.001999 g^2, corrections 0.19 and 0.001999
    p2, _, _ = mlp_ref.adam(p1, m1, v1, g, 2, 1e-3)
    assert np.allclose(p2, p1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
