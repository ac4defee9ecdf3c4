"""Parity of the exact HIP path (tpe_energy / tpe_gradient through the C ABI) with the FP64 oracle.

Tolerances: energy relative error <= 1e-6, gradient max-norm relative error <= 1e-5 (FP32 pair
arithmetic with compensated sums, FP64 finalize and gather).
"""
import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M
from tests.gpu_util import HAVE_GPU, log, needs_gpu, rel_energy, rel_grad_maxnorm, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]

E_TOL = 1e-6
G_TOL = 1e-5


def _patch(X, F, center, nfaces):
    c = X[F].mean(1)
    sel = np.sort(np.argsort(np.linalg.norm(c - center, axis=1), kind="stable")[:nfaces])
    Fs = F[sel]
    used, inv = np.unique(Fs, return_inverse=True)
    return X[used].copy(), inv.reshape(Fs.shape).astype(np.int32)


def small_meshes():
    X, F = M.icosphere(0)
    yield "L0-icosahedron", M.radial_jitter(X, 0.02, 1), F
    X, F = M.icosphere(1)
    yield "L1-jitter", M.radial_jitter(X, 0.01, 0), F
    X, F = M.icosphere(2)
    Xb, _, _ = M.bump(X, 0, 0.3, 0.15)
    yield "L2-bump", Xb, F
    X, F = M.icosphere(3)
    Xb, _, _ = M.bump(X, 0, 0.3, 0.05)
    yield "L3-gap-patch", *_patch(Xb, F, Xb[3] * 0.97, 333)
    X, F = M.icosphere(4)
    yield "L4-sh", M.sh_deform(X, 2, 6, 0.05, 3)[0], F


@pytest.mark.parametrize("name,X,F", list(small_meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_small_meshes_parity(name, X, F):
    T = tpe()
    log("case", name, F.shape[0])
    Eo, Go = oracle.gradient(X, F)
    Xd, Fd = upload(X, F)
    E, G = T.gradient(Xd, Fd)
    E = float(E.cpu()); G = G.cpu().numpy()
    Ee = float(T.energy(Xd, Fd).cpu())
    log(name, "rel E", rel_energy(E, Eo), "rel E(energy kernel)", rel_energy(Ee, Eo), "rel G", rel_grad_maxnorm(G, Go))
    assert rel_energy(E, Eo) <= E_TOL
    assert rel_energy(Ee, Eo) <= E_TOL
    assert rel_grad_maxnorm(G, Go) <= G_TOL


def test_two_triangles_closed_form():
    T = tpe()
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 0, 1], [2, 0, 1], [1, 1, 1]], dtype=np.float64)
    F = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    Xd, Fd = upload(X, F)
    E, G = T.gradient(Xd, Fd)
    assert float(E.cpu()) == pytest.approx(1.0 / 128.0, rel=1e-6)
    assert float(T.energy(Xd, Fd).cpu()) == pytest.approx(1.0 / 128.0, rel=1e-6)
    Eo, Go = oracle.gradient(X, F)
    assert rel_grad_maxnorm(G.cpu().numpy(), Go) <= G_TOL


def test_c1_parity():
    T = tpe()
    c = M.make_config("C1")
    Eo, Go = oracle.gradient(c.X, c.F)
    Xd, Fd = upload(c.X, c.F)
    E, G = T.gradient(Xd, Fd)
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    log("C1 rel E", eE, "rel G", eG)
    assert eE <= E_TOL and eG <= G_TOL


def test_c2_parity():
    T = tpe()
    c = M.make_config("C2")
    log("C2 oracle start", c.nF)
    Eo, Go = oracle.gradient(c.X, c.F)
    Xd, Fd = upload(c.X, c.F)
    E, G = T.gradient(Xd, Fd)
    Ee = T.energy(Xd, Fd)
    eE, eG = rel_energy(float(E.cpu()), Eo), rel_grad_maxnorm(G.cpu().numpy(), Go)
    eEe = rel_energy(float(Ee.cpu()), Eo)
    log("C2 rel E", eE, "rel E(energy kernel)", eEe, "rel G", eG)
    assert eE <= E_TOL and eEe <= E_TOL and eG <= G_TOL


def test_c3_parity_sampled():
    """Level-6 bump at gap 0.02: full oracle energy, oracle gradient at sampled vertices that
    include the closest-approach region (where the gradient is largest)."""
    T = tpe()
    c = M.make_config("C3")
    scale = 1e-4 / 6
    Xd, Fd = upload(c.X, c.F)
    E, G = T.gradient(Xd, Fd, scale=scale)
    G = G.cpu().numpy()
    E = float(E.cpu())
    log("C3 oracle energy start", c.nF)
    Eo = oracle.energy(c.X, c.F, scale=scale)
    rng = np.random.default_rng(0)
    top = np.argsort(-np.abs(G).max(1))[:16]
    verts = np.unique(np.concatenate([top, rng.choice(c.V, 16, replace=False)])).astype(np.int32)
    Go = oracle.gradient_at(c.X, c.F, verts, scale=scale)
    # max-norm relative to the largest gradient component (the closest-approach vertices are sampled)
    eG = float(np.abs(G[verts] - Go).max() / np.abs(Go).max())
    log("C3 rel E", rel_energy(E, Eo), "rel G(sampled)", eG)
    assert rel_energy(E, Eo) <= E_TOL
    assert eG <= G_TOL


@pytest.mark.parametrize("name", ["C4", "C5"])
def test_full_size_sampled_parity(name):
    """The level-7 (327,680 faces) and level-8 (1,310,720 faces, gap 0.01, degree-32 wrinkles)
    workloads in the launch configuration bench.py times: the oracle's gradient at sampled
    vertices (the 8 with the largest gradient -- nearly touching pairs -- and 8 random ones), and
    identities that hold at any size: zero net force and torque, and Euler's identity
    sum (x_v - x0) . G_v = (4 + q - p) E about the largest-gradient vertex x0, each relative to the
    sum of the magnitudes of its terms."""
    T = tpe()
    c = M.make_config(name)
    Xd, Fd = upload(c.X, c.F)
    log(name, "exact start", c.nF)
    E, G = T.gradient(Xd, Fd)
    G = G.cpu().numpy()
    E = float(E.cpu())
    gn = np.abs(G).max(1)
    rng = np.random.default_rng(0)
    verts = np.unique(np.concatenate([np.argsort(-gn)[:8], rng.choice(c.V, 8, replace=False)])).astype(np.int32)
    Go = oracle.gradient_at(c.X, c.F, verts)
    eG = float(np.abs(G[verts] - Go).max() / np.abs(G).max())
    x0 = c.X[np.argmax(gn)]
    terms = ((c.X - x0) * G).sum(1)
    euler = abs(terms.sum() + 2.0 * E) / np.abs(terms).sum()
    force = np.abs(G.sum(0)).max() / np.abs(G).sum()
    torque = np.abs(np.cross(c.X - x0, G).sum(0)).max() / (np.abs(c.X - x0).max() * np.abs(G).sum())
    log(name, "rel G(sampled)", eG, "euler", euler, "force", force, "torque", torque)
    assert eG <= G_TOL
    assert euler <= 1e-6 and force <= 1e-6 and torque <= 1e-6


def test_scaling_and_euler_identity():
    """E(2X) = E(X)/4 and sum_v x_v . G_v = -2 E hold for any mesh (homogeneity of degree 4+q-p)."""
    T = tpe()
    c = M.make_config("C2")
    Xd, Fd = upload(c.X, c.F)
    E1, G1 = T.gradient(Xd, Fd)
    E2, G2 = T.gradient(2 * Xd, Fd)
    E1, E2 = float(E1.cpu()), float(E2.cpu())
    # power-of-two scaling is exact inside the library
    assert E2 == E1 / 4
    assert float((Xd * G1).sum().cpu()) == pytest.approx(-2 * E1, rel=1e-6)
    assert np.abs(G2.cpu().numpy() * 8 - G1.cpu().numpy()).max() == 0.0


def test_rigid_motion_gpu():
    T = tpe()
    c = M.make_config("C1")
    R = M.random_rotation(5)
    Xd, Fd = upload(c.X, c.F)
    Xr, _ = upload(c.X @ R.T + np.array([0.25, -3.0, 1.0]), c.F)
    E1, G1 = T.gradient(Xd, Fd)
    E2, G2 = T.gradient(Xr, Fd)
    assert rel_energy(float(E2.cpu()), float(E1.cpu())) <= 2e-6
    G1 = G1.cpu().numpy(); G2 = G2.cpu().numpy()
    assert rel_grad_maxnorm(G2, G1 @ R.T) <= 2e-5
    # zero net force and torque
    scale = np.abs(G1).max()
    assert np.abs(G1.sum(0)).max() <= 1e-5 * scale
    assert np.abs(np.cross(c.X, G1).sum(0)).max() <= 1e-5 * scale


def test_determinism():
    T = tpe()
    c = M.make_config("C1")
    Xd, Fd = upload(c.X, c.F)
    E1, G1 = T.gradient(Xd, Fd)
    E2, G2 = T.gradient(Xd, Fd)
    assert float(E1.cpu()) == float(E2.cpu())
    assert np.array_equal(G1.cpu().numpy(), G2.cpu().numpy())


@pytest.mark.parametrize("waves", [1, 64, 100000])
def test_split_independence(waves):
    """Different column splits of the pair kernel give the same result within tolerance."""
    T = tpe()
    c = M.make_config("C1")
    Eo, Go = oracle.gradient(c.X, c.F)
    Xd, Fd = upload(c.X, c.F)
    ctx = T.context(Xd.device)
    ctx.set_option(T.OPT_TARGET_WAVES, waves)
    try:
        E, G = T.gradient(Xd, Fd)
    finally:
        ctx.set_option(T.OPT_TARGET_WAVES, 0)
    assert rel_energy(float(E.cpu()), Eo) <= E_TOL
    assert rel_grad_maxnorm(G.cpu().numpy(), Go) <= G_TOL


def _sym_cases():
    X, F = M.icosphere(0)
    yield "L0 (20 faces, one super block)", M.radial_jitter(X, 0.02, 1), F
    X, F = M.icosphere(2)
    yield "L2 (320 faces)", M.radial_jitter(X, 0.02, 2), F
    X, F = M.icosphere(3)
    Xb, _, _ = M.bump(X, 0, 0.3, 0.1)
    yield "L3-bump (1,280 faces, ragged)", Xb, F
    X, F = M.icosphere(4)
    yield "L4-patch (2,001 faces, ragged)", *_patch(M.sh_deform(X, 2, 6, 0.05, 3)[0], F, X[7], 2001)


@pytest.mark.parametrize("name,X,F", list(_sym_cases()), ids=lambda v: v if isinstance(v, str) else "")
@pytest.mark.parametrize("waves", [0, 1, 7, 100000])
@pytest.mark.parametrize("nw", [1, 2, 4, 8])
def test_symmetric_kernel(name, X, F, waves, nw):
    """The symmetric pair kernel (default for (6, 12)) with work-groups of 1, 2, 4 and 8 waves, and
    the row-only kernel, against the oracle, for several work-group counts (uneven ranges, empty ranges,
    one work-group for everything)."""
    T = tpe()
    Eo, Go = oracle.gradient(X, F)
    Xd, Fd = upload(X, F)
    ctx = T.context(Xd.device)
    ctx.set_option(T.OPT_TARGET_WAVES, waves)
    ctx.set_option(T.OPT_SYM_WAVES, nw)
    out = {}
    try:
        for sym in ((1, 0) if nw == 4 else (1,)):
            ctx.set_option(T.OPT_SYMMETRIC, sym)
            E, G = T.gradient(Xd, Fd)
            Ee = T.energy(Xd, Fd)
            out[sym] = (float(E.cpu()), G.cpu().numpy(), float(Ee.cpu()))
    finally:
        ctx.set_option(T.OPT_SYMMETRIC, 1)
        ctx.set_option(T.OPT_TARGET_WAVES, 0)
        ctx.set_option(T.OPT_SYM_WAVES, 0)
    for sym, (E, G, Ee) in out.items():
        eE, eEe, eG = rel_energy(E, Eo), rel_energy(Ee, Eo), rel_grad_maxnorm(G, Go)
        log(name, "waves", waves, "nw", nw, "symmetric", sym, "rel E", eE, "rel E(energy kernel)", eEe, "rel G", eG)
        assert eE <= E_TOL and eEe <= E_TOL and eG <= G_TOL


@pytest.mark.parametrize("name,X,F", list(_sym_cases())[1:], ids=lambda v: v if isinstance(v, str) else "")
def test_symmetric_kernel_without_barriers_gives_the_same_bits(name, X, F):
    """The barrier-free symmetric kernel (2 and 4 waves per work-group) reduces the waves' column
    sums in the same order as the kernel with barriers: energy and gradient bit for bit, for
    several work-group counts (one work-group for everything: the waves drift the furthest)."""
    T = tpe()
    Xd, Fd = upload(X, F)
    ctx = T.context(Xd.device)
    try:
        for nw in (2, 4):
            ctx.set_option(T.OPT_SYM_WAVES, nw)
            for waves in (0, 1, 7):
                ctx.set_option(T.OPT_TARGET_WAVES, waves)
                res = []
                for barriers in (1, 0):
                    ctx.set_option(T.OPT_SYM_BARRIERS, barriers)
                    E, G = T.gradient(Xd, Fd)
                    Ee = T.energy(Xd, Fd)
                    res.append((float(E.cpu()), G.cpu().numpy(), float(Ee.cpu())))
                log(name, "nw", nw, "waves", waves, "E", res[0][0], res[1][0])
                assert res[0][0] == res[1][0] and res[0][2] == res[1][2]
                assert np.array_equal(res[0][1], res[1][1])
    finally:
        ctx.set_option(T.OPT_SYM_BARRIERS, 0)
        ctx.set_option(T.OPT_TARGET_WAVES, 0)
        ctx.set_option(T.OPT_SYM_WAVES, 0)


def test_exact_plan_reports_the_kernel_choice():
    """tpe_exact_plan: by default the barrier-free kernel with 4 waves per work-group (8 where the
    partials of 4 would exceed 64 GiB); with barriers
    the fewest waves whose column partials fit in 8 GiB; the partial bytes of the schedule (8 sums x
    64 columns x 4 bytes per symmetric unit); the row-only kernel when the symmetric one is off."""
    T = tpe()
    import torch
    ctx = T.context(torch.device("cuda", 0))

    def colpart(nF, nw):
        sb = 128 * nw
        fp = -(-nF // sb) * sb
        nsb, nch, sbc = fp // sb, fp // 64, 2 * nw
        return (nsb * (nch - sbc) - sbc * nsb * (nsb - 1) // 2) * 8 * 64 * 4

    sizes = (20480, 262144, 327680, 370688, 400000, 1310720)
    for nF, nw in zip(sizes + (1500000, 2000000), (4, 4, 4, 4, 4, 4, 8, 8)):  # 8 beyond 64 GiB at 4
        sym, w, cp, scratch = ctx.exact_plan(nF, nF // 2 + 2, True)
        log("plan", nF, sym, w, cp, scratch)
        assert sym == 2 and w == nw and cp == colpart(nF, nw) and scratch > cp
    try:
        ctx.set_option(T.OPT_SYM_BARRIERS, 1)
        for nF, nw in zip(sizes, (1, 1, 2, 2, 4, 4)):
            sym, w, cp, _ = ctx.exact_plan(nF, nF // 2 + 2, True)
            assert sym == 1 and w == nw and cp == colpart(nF, nw)
        ctx.set_option(T.OPT_SYM_BARRIERS, 0)
        ctx.set_option(T.OPT_SYM_WAVES, 1)
        assert ctx.exact_plan(20480, 10242, True)[:3] == (1, 1, colpart(20480, 1))  # one wave: no barrier to drop
        ctx.set_option(T.OPT_SYM_WAVES, 2)
        assert ctx.exact_plan(20480, 10242, True)[:3] == (2, 2, colpart(20480, 2))
        ctx.set_option(T.OPT_SYMMETRIC, 0)
        assert ctx.exact_plan(20480, 10242, True)[:3] == (0, 0, 0)
    finally:
        ctx.set_option(T.OPT_SYM_BARRIERS, 0)
        ctx.set_option(T.OPT_SYM_WAVES, 0)
        ctx.set_option(T.OPT_SYMMETRIC, 1)


def test_symmetric_waves_option_rejects_other_values():
    T = tpe()
    import torch
    ctx = T.context(torch.device("cuda", 0))
    for bad in (3, 16, -1):
        with pytest.raises(T.TPEError):
            ctx.set_option(T.OPT_SYM_WAVES, bad)


def test_pair_count():
    T = tpe()
    for level in (1, 3, 5):
        X, F = M.icosphere(level)
        _, Fd = upload(X, F)
        nF = F.shape[0]
        assert T.pair_count(Fd, X.shape[0]) == nF * nF - 13 * nF + 60
    X, F = M.icosphere(2)
    _, Fd = upload(X, F)
    assert T.pair_count(Fd, X.shape[0]) == oracle.pair_count(F)


def test_unreferenced_vertices_and_face_order():
    """Extra vertices get zero gradient; permuting faces does not change the result."""
    T = tpe()
    c = M.make_config("C1")
    X = np.concatenate([c.X, np.array([[5.0, 5.0, 5.0]])], 0)
    F = c.F[np.random.default_rng(2).permutation(c.nF)]
    Eo, Go = oracle.gradient(X, F)
    Xd, Fd = upload(X, F)
    E, G = T.gradient(Xd, Fd)
    G = G.cpu().numpy()
    assert np.all(G[-1] == 0.0)
    assert rel_energy(float(E.cpu()), Eo) <= E_TOL
    assert rel_grad_maxnorm(G, Go) <= G_TOL


def test_error_paths():
    T = tpe()
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 0, 1], [2, 0, 1], [1, 1, 1]], dtype=np.float64)
    F = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    Xd, Fd = upload(X, F)
    with pytest.raises(T.TPEError) as e:
        T.gradient(Xd, upload(X, np.array([[0, 1, 2], [3, 4, 9]], dtype=np.int32))[1])
    assert e.value.code == -1
    Xdeg = X.copy(); Xdeg[5] = Xdeg[4]
    with pytest.raises(T.TPEError) as e:
        T.gradient(upload(Xdeg, F)[0], Fd)
    assert e.value.code == -2
    Xnan = X.copy(); Xnan[0, 0] = np.nan
    with pytest.raises(T.TPEError) as e:
        T.energy(upload(Xnan, F)[0], Fd)
    assert e.value.code == -3
    Xc = np.concatenate([X[:3], X[:3][:, [1, 0, 2]]], 0)
    with pytest.raises(T.TPEError) as e:
        T.gradient(upload(Xc, F)[0], Fd)
    assert e.value.code == -3
    with pytest.raises(T.TPEError) as e:
        T.energy(Xd, Fd, q=4.0, p=10.0)
    assert e.value.code == -6
    with pytest.raises(T.TPEError) as e:
        T.energy(Xd, Fd, q=6.0, p=5.0)
    assert e.value.code == -1
    # the context keeps working after errors
    E = T.energy(Xd, Fd)
    assert float(E.cpu()) == pytest.approx(1.0 / 128.0, rel=1e-6)
