"""BF16-MFMA MLP kernels (forward, hand-written backward, Adam, checkpoint) vs the FP64 reference."""
import os

import numpy as np
import pytest

from oracle import mlp_ref
from tests.gpu_util import log, needs_gpu, tpe

pytestmark = [pytest.mark.gpu, needs_gpu]


def batch(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 32)).astype(np.float32)
    T = np.zeros((n, 16), np.float32)
    T[:, :7] = rng.normal(size=(n, 7))
    T[:, 15] = rng.uniform(0.5, 1.5, n)
    T[n - 7:, 15] = 0.0  # unused rows
    return X, T


def test_forward_matches_fp64_reference():
    import torch
    T_ = tpe()
    m = T_.MLP(seed=3)
    p = m.get_params()
    assert p.size == 11472
    for n in (1, 31, 32, 1000):
        X, _ = batch(n, n)
        Y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy()
        Yr, _ = mlp_ref.forward(p, X.astype(np.float64))
        err = np.abs(Y - Yr).max() / np.abs(Yr).max()
        log("mlp forward n", n, "rel err", err)
        assert err < 2e-2


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_backward_matches_fp64_reference(lam):
    import torch
    T_ = tpe()
    m = T_.MLP(seed=5)
    m.set_smoothness(lam)  # difference term over consecutive rows of each 32-row tile
    p = m.get_params()
    X, T = batch(777, 1)
    g = m.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()).cpu().numpy()
    gr = mlp_ref.gradient(p, X.astype(np.float64), T.astype(np.float64), lam=lam, tile=32)
    # Tolerance: every product takes BF16 operands (unit roundoff 2^-9) and the input-layer
    # gradient passes through three chained products that sum 16..777 terms with cancellation,
    # so max-norm errors of a few percent are expected; an indexing or transposition mistake
    # gives O(1) errors.
    offs = np.cumsum([0] + [int(np.prod(s)) for s in mlp_ref.SHAPES])
    errs = []
    for i in range(len(mlp_ref.SHAPES)):
        a, b = offs[i], offs[i + 1]
        errs.append(np.abs(g[a:b] - gr[a:b]).max() / max(np.abs(gr[a:b]).max(), 1e-12))
        log("mlp grad block", i, mlp_ref.SHAPES[i], "rel err", errs[-1])
    assert max(errs) < 0.1
    # and the whole gradient direction agrees closely
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    log("mlp grad cosine", cos)
    assert cos > 0.999


def test_training_reduces_loss_and_checkpoint_roundtrip(tmp_path):
    import torch
    T_ = tpe()
    rng = np.random.default_rng(2)
    X = rng.normal(size=(4096, 32)).astype(np.float32)
    A = rng.normal(size=(32, 7)) / 6
    T = np.zeros((4096, 16), np.float32)
    T[:, :7] = np.tanh(X @ A) + 0.1 * (X[:, :7] ** 2)
    T[:, 15] = 1.0
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m = T_.MLP(seed=11)
    losses = []
    for it in range(300):
        losses.append(float(m.train_step(Xd, Td, 3e-3)))
    log("mlp loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    # the reported loss is the reference loss of the parameters before the step
    path = str(tmp_path / "mlp.bin")
    m.set_gate(0.17)
    m.save(path)
    m2 = T_.MLP.load(path)
    assert np.array_equal(m.get_params(), m2.get_params())
    assert m2.gate() == np.float32(0.17)
    # a checkpoint of the first format (no gate field) loads with gate 0
    raw = open(path, "rb").read()
    assert raw[:8] == b"TPEMLP02"
    v1 = str(tmp_path / "mlp_v1.bin")
    with open(v1, "wb") as f:
        f.write(b"TPEMLP01" + raw[8:32] + raw[40:])
    m3 = T_.MLP.load(v1)
    assert m3.gate() == 0.0 and np.array_equal(m.get_params(), m3.get_params())
    m.set_gate(0.0)
    m2.set_gate(0.0)
    l1 = [float(m.train_step(Xd, Td, 3e-3)) for _ in range(5)]
    l2 = [float(m2.train_step(Xd, Td, 3e-3)) for _ in range(5)]
    assert l1 == l2  # resumed Adam state is exact and the kernels are deterministic
    p = m.get_params()
    ref = mlp_ref.loss(p, X.astype(np.float64), T.astype(np.float64))
    now = float(m.train_step(Xd, Td, 1e-12))
    assert abs(now - ref) / ref < 5e-2
