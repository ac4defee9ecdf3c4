"""FP64 NumPy reference of the far-field correction network (32-64-64-64-16, ReLU).

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


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    assert o == p.size
    return out


def forward(p, X):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    Z3 = H2 @ W3 + b3
    H3 = np.maximum(Z3, 0.0)
    Y = H3 @ W4 + b4
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


def gradient(p, X, T, lam=0.0, tile=32):
    """Backpropagation of loss() by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    Y, (X, Z1, H1, Z2, H2, Z3, H3) = forward(p, X)
    w = T[:, 15]
    d = (Y - T)[:, :N_USED]
    g = 2.0 * w[:, None] * d
    if lam:
        m = _pairs(len(w), tile)
        vD = (w[m] * w[m + 1])[:, None] * (d[m + 1] - d[m])
        np.add.at(g, m + 1, 2.0 * lam * vD)
        np.add.at(g, m, -2.0 * lam * vD)
    dY = np.zeros_like(Y)
    dY[:, :N_USED] = g / (N_USED * w.sum())
    gW4 = H3.T @ dY; gb4 = dY.sum(0)
    dZ3 = (dY @ W4.T) * (Z3 > 0)
    gW3 = H2.T @ dZ3; gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3.T) * (Z2 > 0)
    gW2 = H1.T @ dZ2; gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * (Z1 > 0)
    gW1 = X.T @ dZ1; gb1 = dZ1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
