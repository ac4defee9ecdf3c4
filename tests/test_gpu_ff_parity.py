"""The cluster approximations on the GPU against the FP64 oracle of the same scheme
(oracle/tpe_oracle_ff.c; paper Sec. 3.2), element by element, at theta > 0.

- tree order: integer work, bit-exact;
- tpe_farfield (clustered inner integrals): energy <= 1e-6 relative, gradient max-norm <= 1e-5
  relative, and the walk's interaction counts equal (they are integer outcomes of the FP32
  admissibility decisions, which both sides take the same way);
- tpe_farfield_dual: the same bounds on the energy and on the gradient at sampled vertices, and the
  list counts equal;
- tpe_farfield_samples: the same selected (block, cluster) pairs, features and targets to FP32
  accuracy (see the tolerances below).
"""
import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M
from tests.gpu_util import log, needs_gpu, rel_energy, rel_grad_maxnorm, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]


def _mesh(name):
    if name == "L3":
        c = M.make_config("C1")
        return c.X, c.F
    if name == "L4":
        X, F = M.icosphere(4)
        return M.sh_deform(X, 2, 8, 0.05, 0)[0], F
    c = M.make_config("C2")
    return c.X, c.F


@pytest.mark.parametrize("name,leaf", [("L3", 32), ("L3", 1), ("L4", 32), ("L4", 7), ("C2", 32)])
def test_tree_order_is_the_oracles(name, leaf):
    T = tpe()
    X, F = _mesh(name)
    log("tree order", name, "leaf", leaf, "faces", F.shape[0])
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=leaf)
    got = tree.order().cpu().numpy().view(np.uint32)
    want = oracle.kd_order(X, F, leaf)
    assert np.array_equal(got, want), int((got != want).sum())


@pytest.mark.parametrize("name,theta", [("L3", 1.0), ("L4", 0.5), ("L4", 1.0), ("C2", 0.5), ("C2", 0.25)])
def test_farfield_is_the_oracles(name, theta):
    T = tpe()
    X, F = _mesh(name)
    log("farfield", name, "theta", theta)
    Eo, Go, so = oracle.farfield(X, F, theta, leaf=32)
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=32)
    E, G = T.farfield(tree, Xd, Fd, theta=theta)
    st = T.context(Xd.device).farfield_stats()
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log("  stats gpu", st, "oracle", so, "rel E", eE, "rel G", eG)
    assert so[0] > 0  # far clusters were used
    assert tuple(st) == tuple(so)
    assert eE <= 1e-6 and eG <= 1e-5
    # the heaviest-first launch order of the next monopole call computes the same bits
    E2, G2 = T.farfield(tree, Xd, Fd, theta=theta)
    assert float(E2.cpu()) == float(E.cpu()) and np.array_equal(G2.cpu().numpy(), G.cpu().numpy())


def _ragged_patch():
    """An open patch of 2,001 faces cut from a deformed level-4 sphere (the faces nearest one
    vertex): the last leaf is short, and the near pieces and tiles have odd lengths."""
    X, F = M.icosphere(4)
    X = M.sh_deform(X, 2, 6, 0.05, 3)[0]
    c = X[F].mean(1)
    sel = np.sort(np.argsort(np.linalg.norm(c - X[7], axis=1), kind="stable")[:2001])
    used, inv = np.unique(F[sel], return_inverse=True)
    return X[used].copy(), inv.reshape(-1, 3).astype(np.int32)


@pytest.mark.parametrize("leaf", [32, 7])
def test_farfield_on_a_ragged_open_patch_is_the_oracles(leaf):
    T = tpe()
    X, F = _ragged_patch()
    log("farfield ragged patch", F.shape[0], "faces, leaf", leaf)
    Eo, Go, so = oracle.farfield(X, F, 0.5, leaf=leaf)
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=leaf)
    E, G = T.farfield(tree, Xd, Fd, theta=0.5)
    st = T.context(Xd.device).farfield_stats()
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log("  stats gpu", st, "oracle", so, "rel E", eE, "rel G", eG)
    assert so[0] > 0 and tuple(st) == tuple(so)
    assert eE <= 1e-6 and eG <= 1e-5


@pytest.mark.parametrize("name,theta,nsample", [("L3", 1.0, 0), ("L4", 0.5, 96), ("C2", 0.5, 48)])
def test_farfield_dual_is_the_oracles(name, theta, nsample):
    T = tpe()
    X, F = _mesh(name)
    log("dual", name, "theta", theta)
    verts = None if nsample == 0 else np.random.default_rng(1).choice(X.shape[0], nsample, replace=False)
    Eo, Go, so = oracle.farfield_dual(X, F, theta, leaf=32, verts=verts)
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=32)
    E, G = T.farfield_dual(tree, Xd, Fd, theta=theta)
    st = T.context(Xd.device).farfield_stats()
    G = G.cpu().numpy()
    if verts is not None:
        G = G[verts]
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G, Go)
    log("  stats gpu", st[:2], "oracle", so, "rel E", eE, "rel G", eG)
    assert so[0] > 0
    assert tuple(st[:2]) == tuple(so)
    assert eE <= 1e-6 and eG <= 1e-5


def test_farfield_and_dual_at_level_7_are_the_oracles():
    """The level-7 workload of the far-field timing (327,680 faces, theta 0.5, leaves of 32):
    the monopole far field element by element against the FP64 oracle of the scheme (every
    vertex; about 8 s of oracle on 8 host threads), and the dual tree's energy and gradient at 32
    sampled vertices (about 45 s of oracle: its energy needs every pair of the lists)."""
    T = tpe()
    c = M.make_config("C4")
    X, F = c.X, c.F
    perm = oracle.kd_order(X, F, 32)
    log("level 7: oracle far field")
    Eo, Go, so = oracle.farfield(X, F, 0.5, leaf=32, perm=perm)
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=32)
    assert np.array_equal(tree.order().cpu().numpy().view(np.uint32), perm)
    E, G = T.farfield(tree, Xd, Fd, theta=0.5)
    st = T.context(Xd.device).farfield_stats()
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log("  far field: stats gpu", st, "oracle", so, "rel E", eE, "rel G", eG)
    assert tuple(st) == tuple(so)
    assert eE <= 1e-6 and eG <= 1e-5
    verts = np.random.default_rng(1).choice(X.shape[0], 32, replace=False)
    log("level 7: oracle dual tree")
    Eo, Go, so = oracle.farfield_dual(X, F, 0.5, leaf=32, perm=perm, verts=verts)
    E, G = T.farfield_dual(tree, Xd, Fd, theta=0.5)
    st = T.context(Xd.device).farfield_stats()
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy()[verts], Go)
    log("  dual: stats gpu", st[:2], "oracle", so, "rel E", eE, "rel G", eG)
    assert tuple(st[:2]) == tuple(so)
    assert eE <= 1e-6 and eG <= 1e-5


# Tolerances of the samples.  Features are dimensionless FP32 quantities of size <= 4 built from
# FP32 centroids (relative rounding 2^-24 of coordinates <= 1 against distances >= 0.05 in the
# kernels' frame) and FP32 moments: 2e-5 absolute, except where n_S is nearly parallel to e1 and
# the frame's e2 is the normalised difference of nearly equal vectors.  Targets are differences
# (exact - monopole) of FP32 sums of up to 2^20 pair terms whose size is O(1) in the units; each
# term carries a relative error of about p 2^-24 |c| / rho <= 12 * 6e-8 / 0.05 = 1.4e-5: 1e-4.
FEAT_TOL, TARG_TOL = 2e-5, 1e-4


@pytest.mark.parametrize("name", ["L4", "C2"])
def test_farfield_samples_are_the_oracles(name):
    T = tpe()
    X, F = _mesh(name)
    log("samples", name)
    seed, prob, theta = 5, 0.05, 0.5
    so = oracle.farfield_samples(X, F, theta, seed=seed, select_prob=prob, max_faces=1 << 20)
    nb = (F.shape[0] + 63) // 64
    count = np.bincount(so["block"], minlength=nb)
    quota = int(count.max()) + 1  # one free slot per block: the GPU takes every selected cluster
    Xd, Fd = upload(X, F)
    tree = T.build_tree(Xd, Fd, leaf=32)
    f, t = T.farfield_samples(tree, Xd, Fd, theta=theta, seed=seed, select_prob=prob, quota=quota,
                              max_cluster_faces=1 << 20)
    f = f.cpu().numpy().reshape(nb, quota, 64, 32)
    t = t.cpu().numpy().reshape(nb, quota, 64, 16)
    used = t[:, :, 0, 15] > 0
    assert np.array_equal(used.sum(1), count)
    assert not used[:, -1].any()
    assert np.all(f[:, :, :, 19:] == 0)
    index = {(int(b), int(n)): k for k, (b, n) in enumerate(zip(so["block"], so["node"]))}
    worst_f, worst_t, nrows = 0.0, 0.0, 0
    ff_all, tt_all = [], []
    for b in range(nb):
        for c in range(int(count[b])):
            node = int(t[b, c, 0, 14])
            k = index.pop((b, node))  # KeyError: a cluster the oracle did not select
            w = so["targets"][k, :, 7] > 0
            assert np.array_equal(t[b, c, :, 15] > 0, w)
            ff_all.append(np.abs(f[b, c, w, :19] - so["feats"][k, w]))
            tt_all.append(np.abs(t[b, c, w, :7] - so["targets"][k, w, :7]))
            nrows += int(w.sum())
    assert not index  # every cluster the oracle selected was sampled
    ff = np.concatenate(ff_all)
    tt = np.concatenate(tt_all)
    log("  rows", nrows, "feature err max", ff.max(), "p99.9", np.quantile(ff.max(1), 0.999),
        "target err max", tt.max(), "p99.9", np.quantile(tt.max(1), 0.999))
    # the frame's e2 degrades where n_S is nearly parallel to e1 (|n_S . e2| small): allow it there
    ok = ff.max(1) <= FEAT_TOL
    assert ok.mean() >= 0.999, ok.mean()
    assert tt.max() <= TARG_TOL
