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
    """Against the reference with the kernels' operand rounding (BF16 operands, FP32 activations):
    the remaining differences are the FP32 summation of exact BF16 products (relative 1e-7 of a
    layer's sums) -- and, where such a difference moves an activation across a BF16 rounding
    boundary (probability ~1e-4 per activation), one BF16 step (2^-8 relative) of that activation,
    which reaches the outputs through one row of weights.  The FP64 network is the accuracy report."""
    import torch
    T_ = tpe()
    m = T_.MLP(seed=3)
    p = m.get_params()
    assert p.size == 11472
    for n in (1, 31, 32, 1000, 8192):
        X, _ = batch(n, n)
        Y = m.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        Yb, _ = mlp_ref.forward(p, X.astype(np.float64), low=True)
        Yr, _ = mlp_ref.forward(p, X.astype(np.float64))
        scale = np.abs(Yb).max()
        row = np.abs(Y - Yb).max(1) / scale
        err64 = np.abs(Y - Yr).max() / np.abs(Yr).max()
        log("mlp forward n", n, "vs BF16-rounding reference: max", row.max(), "median", np.median(row),
            "rows within 1e-4:", (row <= 1e-4).mean(), "| vs FP64", err64)
        assert (row <= 1e-4).mean() >= 0.99
        assert row.max() <= 1e-2
        assert err64 < 2e-2


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_backward_matches_fp64_reference(lam):
    """The hand-written backward pass against the reference with the kernels' rounding, per
    parameter block: max-norm error (relative to the block's largest entry) <= 1e-3, relative L2
    error <= 1e-4, and <= 3e-4 for the first layer's weights.  The kernel sums exact BF16 products
    in FP32, the reference exactly; the back-propagated errors are sums of 64 terms of both signs,
    so their FP32 values can differ from the exact ones by 1e-6 and more of their size, and where
    that moves one across a BF16 rounding boundary before the next product, one term of a gradient
    sum changes by one BF16 step (2^-8 of the term).  The first layer's weight gradient sits at
    the end of three such chains and collects most of these crossings (measured L2 1.1e-4 and
    1.3e-4 for the two cases, every other block <= 3.4e-5).  An indexing or transposition mistake
    gives O(1) errors on every measure.  The FP64 gradient is the accuracy report (BF16 operands
    through three chained products: a few percent per block)."""
    import torch
    T_ = tpe()
    m = T_.MLP(seed=5)
    m.set_smoothness(lam)  # difference term over consecutive rows of each 32-row tile
    p = m.get_params()
    X, T = batch(777, 1)
    g = m.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()).cpu().numpy().astype(np.float64)
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    gb = mlp_ref.gradient(p, X64, T64, lam=lam, tile=32, low=True)
    gr = mlp_ref.gradient(p, X64, T64, lam=lam, tile=32)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in mlp_ref.SHAPES])
    errs, errs2, errs64 = [], [], []
    for i in range(len(mlp_ref.SHAPES)):
        a, b = offs[i], offs[i + 1]
        errs.append(np.abs(g[a:b] - gb[a:b]).max() / max(np.abs(gb[a:b]).max(), 1e-30))
        errs2.append(np.linalg.norm(g[a:b] - gb[a:b]) / max(np.linalg.norm(gb[a:b]), 1e-30))
        errs64.append(np.abs(g[a:b] - gr[a:b]).max() / max(np.abs(gr[a:b]).max(), 1e-30))
        log("mlp grad block", i, mlp_ref.SHAPES[i], "vs BF16-rounding reference: max", errs[-1], "L2", errs2[-1],
            "| vs FP64", errs64[-1])
    assert errs2[0] <= 3e-4 and max(errs2[1:]) <= 1e-4
    assert max(errs) <= 1e-3
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    log("mlp grad cosine with the FP64 gradient", cos)
    assert cos > 0.999


def _checkpoint(path):
    """(step, gate, P, M, V) of a TPEMLP02 checkpoint."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"TPEMLP02"
    step = int(np.frombuffer(raw[24:32], np.int64)[0])
    gate = float(np.frombuffer(raw[32:36], np.float32)[0])
    body = np.frombuffer(raw[40:], np.float32)
    n = body.size // 3
    return step, gate, body[:n].astype(np.float64), body[n:2 * n].astype(np.float64), body[2 * n:].astype(np.float64)


def test_adam_steps_match_numpy_adam(tmp_path):
    """Two training steps against NumPy Adam fed with the kernel's own gradient of each step
    (tpe_mlp_gradient on the same batch: the same tiles summed in the same order): parameters and
    both moments, read back from checkpoints, agree to FP32 rounding (1e-6 relative)."""
    import torch
    T_ = tpe()
    m = T_.MLP(seed=9)
    X, T = batch(1000, 4)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p = m.get_params().astype(np.float64)
    mo, vo = np.zeros_like(p), np.zeros_like(p)
    for step, lr in ((1, 1e-3), (2, 5e-4)):
        g = m.gradient(Xd, Td).cpu().numpy().astype(np.float64)
        m.train_step(Xd, Td, lr)
        p, mo, vo = mlp_ref.adam(p, mo, vo, g, step, lr)
        path = str(tmp_path / f"adam{step}.bin")
        m.save(path)
        st, _, P, M_, V_ = _checkpoint(path)
        assert st == step
        for name, got, want in (("params", P, p), ("m", M_, mo), ("v", V_, vo)):
            err = np.abs(got - want).max() / np.abs(want).max()
            log("adam step", step, name, "rel err", err)
            assert err <= 1e-6
        p, mo, vo = P, M_, V_  # continue from the kernel's FP32 state


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
