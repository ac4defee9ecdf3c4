"""FP64 NumPy reference of the far-field correction network (32-64-64-64-16, ReLU), exact or with
the operand rounding of BF16 matrix-core kernels (low=True), and one Adam step.

TEST INFRASTRUCTURE ONLY: used by tests to check the BF16-MFMA forward and hand-written backward
kernels of the library; never imported by the product path.  Parameter layout (one flat vector):
W1[32][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64][16], b4[16] (row-major [in][out]).
Loss: [sum_i w_i sum_{j<7} (y_ij - t_ij)^2
        + lam sum_{i, i+1 in one tile} w_i w_{i+1} sum_{j<7} ((y_{i+1,j} - y_ij) - (t_{i+1,j} - t_ij))^2]
      / (7 sum_i w_i),
w_i = target column 15, tiles = consecutive runs of `tile` rows (the second term compares the
differences of the outputs of neighbouring rows with those of the targets).
"""
import numpy as np

SHAPES = [(32, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64, 16), (16,)]
N_USED = 7


def f32(a):
    """Round to the nearest FP32 value (returned as float64)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16(a):
    """Round to the nearest BF16 value, ties to even, through FP32 as a kernel holding FP32 values
    converts them (returned as float64): BF16 keeps the sign, the 8 exponent bits and the top 7
    mantissa bits of an FP32 number."""
    u = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32)).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32).astype(np.float64)


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    assert o == p.size
    return out


def forward(p, X, low=False, rnd=bf16, store=f32):
    """Network outputs Y [n, 16] and the intermediates.  low: the operand rounding of the BF16
    matrix-core kernels -- every product takes operands rounded by `rnd` (BF16) from the values the
    kernel holds, activations are held as `store` (FP32) values, products are summed exactly here
    (the kernels sum them in FP32) and biases are added unrounded."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    if not low:
        rnd = store = _ident
    Z1 = rnd(X) @ rnd(W1) + b1
    H1 = store(np.maximum(Z1, 0.0))
    Z2 = rnd(H1) @ rnd(W2) + b2
    H2 = store(np.maximum(Z2, 0.0))
    Z3 = rnd(H2) @ rnd(W3) + b3
    H3 = store(np.maximum(Z3, 0.0))
    Y = store(rnd(H3) @ rnd(W4) + b4)
    return Y, (X, Z1, H1, Z2, H2, Z3, H3)


def _pairs(n, tile):
    """Indices m of the row pairs (m, m + 1) that lie in one tile."""
    m = np.arange(max(n - 1, 0))
    return m[(m // tile) == ((m + 1) // tile)]


def loss(p, X, T, lam=0.0, tile=32):
    Y, _ = forward(p, X)
    w = T[:, 15]
    d = (Y - T)[:, :N_USED]
    total = (w[:, None] * d * d).sum()
    if lam:
        m = _pairs(len(w), tile)
        D = d[m + 1] - d[m]  # (y_{m+1} - y_m) - (t_{m+1} - t_m)
        total += lam * ((w[m] * w[m + 1])[:, None] * D * D).sum()
    return float(total / (N_USED * w.sum()))


def gradient(p, X, T, lam=0.0, tile=32, low=False, rnd=bf16, store=f32):
    """Backpropagation of loss() by the chain rule, layer by layer.  low: with the kernels'
    rounding (see forward): the per-sample output gradient 2 w (y - t) is formed unnormalised and
    rounded like any operand, each back-propagated error is held as a `store` value and rounded by
    `rnd` where it enters a product, bias gradients are unrounded sums, and the normalisation
    1 / (7 sum w) is applied last."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    Y, (X, Z1, H1, Z2, H2, Z3, H3) = forward(p, X, low, rnd, store)
    if not low:
        rnd = store = _ident
    w = T[:, 15]
    d = (Y - T)[:, :N_USED]
    g = 2.0 * w[:, None] * d
    if lam:
        m = _pairs(len(w), tile)
        vD = (w[m] * w[m + 1])[:, None] * (d[m + 1] - d[m])
        np.add.at(g, m + 1, 2.0 * lam * vD)
        np.add.at(g, m, -2.0 * lam * vD)
    dY = np.zeros_like(Y)
    dY[:, :N_USED] = store(g)
    gW4 = rnd(H3).T @ rnd(dY); gb4 = dY.sum(0)
    dZ3 = store((rnd(dY) @ rnd(W4).T) * (Z3 > 0))
    gW3 = rnd(H2).T @ rnd(dZ3); gb3 = dZ3.sum(0)
    dZ2 = store((rnd(dZ3) @ rnd(W3).T) * (Z2 > 0))
    gW2 = rnd(H1).T @ rnd(dZ2); gb2 = dZ2.sum(0)
    dZ1 = store((rnd(dZ2) @ rnd(W2).T) * (Z1 > 0))
    gW1 = rnd(X).T @ rnd(dZ1); gb1 = dZ1.sum(0)
    full = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return full / (N_USED * w.sum())


def adam(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on parameters p with moments (m, v), gradient g and the
    1-based step count: returns the new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
