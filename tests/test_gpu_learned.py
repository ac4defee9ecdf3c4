"""Learned far-field correction: training samples, fused BF16-MFMA inference in the tree walk,
and the gain over the plain monopole (judged against the exact path)."""
import time

import numpy as np
import pytest

from paper_2509_22110_amd import meshes as M
from tests.gpu_util import log, needs_gpu, rel_energy, rel_grad_maxnorm, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module")
def trained():
    """A network trained in-test on seeded training shapes (seeds 1000..1039, validation
    1040..1045, all disjoint from the evaluation seed 0), on per-output normalized targets, with
    the neighbouring-face difference term at weight 1."""
    tpe()
    from paper_2509_22110_amd import mlp_train as MT
    t0 = time.time()
    X, Y = MT.collect(range(1000, 1040))
    Xv, Yv = MT.collect(range(1040, 1046))
    m = MT.fit(X, Y, Xv, Yv, epochs=8, seed=7, log=log, lam=1.0)
    ratio = MT.per_output_ratio(m, Xv, Yv)
    log(f"trained on {X.shape[0]} samples in {time.time() - t0:.1f} s; validation error / zero-correction "
        f"error per output {np.round(ratio, 3)}")
    return m, ratio


def test_samples_are_finite_and_deterministic():
    import torch
    T = tpe()
    c = M.make_config("C2")  # the level-3 mesh is too coarse to have admissible clusters at theta 0.5
    Xd, Fd = upload(c.X, c.F)
    tree = T.build_tree(Xd, Fd)
    f1, t1 = T.farfield_samples(tree, Xd, Fd, seed=3, select_prob=0.05, quota=8)
    f2, t2 = T.farfield_samples(tree, Xd, Fd, seed=3, select_prob=0.05, quota=8)
    assert torch.equal(f1, f2) and torch.equal(t1, t2)
    keep = t1[:, 15] > 0
    assert int(keep.sum()) > 0
    assert bool(torch.isfinite(f1[keep]).all()) and bool(torch.isfinite(t1[keep]).all())
    # features are rotation-invariant by construction
    R = M.random_rotation(4)
    Xr, _ = upload(c.X @ R.T, c.F)
    tree_r = T.build_tree(Xr, Fd)
    f3, t3 = T.farfield_samples(tree_r, Xr, Fd, seed=3, select_prob=0.05, quota=8)
    k3 = t3[:, 15] > 0
    # same statistics (the k-d order can differ after rotation, so compare distributions)
    a = f1[keep][:, :19].mean(0).cpu().numpy(); b = f3[k3][:, :19].mean(0).cpu().numpy()
    log("feature means", a[:7], b[:7])
    assert np.abs(a[:3] - b[:3]).max() < 0.05


def test_fused_inference_matches_standalone(trained):
    """The network evaluated inside the tree walk gives exactly what tpe_mlp_forward gives on
    the same features."""
    import torch
    m, _ = trained
    T = tpe()
    c = M.make_config("C2")
    Xd, Fd = upload(c.X, c.F)
    tree = T.build_tree(Xd, Fd)
    f, t, p = T.farfield_samples(tree, Xd, Fd, seed=9, select_prob=0.05, quota=8, mlp=m)
    keep = t[:, 15] > 0
    ps = m.forward(f[keep])
    assert torch.equal(p[keep][:, :7], ps[:, :7])


def test_learned_correction_gain(trained):
    """What the trained network gains over the plain monopole, judged against the exact path.

    Measured: on the level-5 workload the correction lowers the energy error 6-9x and the
    gradient's max-norm error about 1.5x.  On the level-7 workload the gradient error stays within
    the 1e-3 target, at the monopole's level (the correction's errors vary from face to face and do
    not cancel at shared vertices the way the monopole's smooth error does); the level-7 energy
    error, a sum over ~1e8 far interactions whose monopole error has a mean of a few percent of
    its spread, moves by whatever small bias the network has there (1.2e-2 to 3e-3 vs the
    monopole's 1.4e-2 between trainings), so it is reported, not asserted."""
    m, ratio = trained
    # every output of the correction beats predicting zero (= the plain monopole) per sample
    assert ratio.max() < 0.5 and ratio.mean() < 0.25
    T = tpe()
    res = {}
    for name in ("C2", "C4"):
        c = M.make_config(name)
        Xd, Fd = upload(c.X, c.F)
        E0, G0 = T.gradient(Xd, Fd)
        E0 = float(E0.cpu()); G0 = G0.cpu().numpy()
        tree = T.build_tree(Xd, Fd)
        Em, Gm = T.farfield(tree, Xd, Fd, theta=0.5)
        El, Gl = T.farfield(tree, Xd, Fd, theta=0.5, mlp=m)
        em = (rel_energy(float(Em.cpu()), E0), rel_grad_maxnorm(Gm.cpu().numpy(), G0))
        el = (rel_energy(float(El.cpu()), E0), rel_grad_maxnorm(Gl.cpu().numpy(), G0))
        res[name] = (em, el)
        log(f"{name}: monopole rel E {em[0]:.3e} rel G {em[1]:.3e} | learned rel E {el[0]:.3e} rel G {el[1]:.3e}")
    (em, el) = res["C2"]
    assert el[0] < 0.5 * em[0]      # energy: at least 2x closer to exact
    assert el[1] < em[1]            # gradient: closer to exact
    (em4, el4) = res["C4"]
    assert em4[1] <= 1e-3 and el4[1] <= 1e-3  # both meet the level-7 gradient target


def test_farfield_speed_and_accuracy_at_c4(trained):
    """Level-7 workload: monopole far field >= 10x faster than the exact kernel at <= 1e-3 gradient
    error; the learned variant's time and error are reported."""
    import torch
    m, _ = trained
    T = tpe()
    c = M.make_config("C4")
    Xd, Fd = upload(c.X, c.F)
    tree = T.build_tree(Xd, Fd)
    def timed(fn):
        fn(); torch.cuda.synchronize()
        t0 = time.perf_counter(); out = fn(); torch.cuda.synchronize()
        return time.perf_counter() - t0, out
    t_e, (E0, G0) = timed(lambda: T.gradient(Xd, Fd))
    t_m, (Em, Gm) = timed(lambda: T.farfield(tree, Xd, Fd, theta=0.5))
    t_l, (El, Gl) = timed(lambda: T.farfield(tree, Xd, Fd, theta=0.5, mlp=m))
    G0 = G0.cpu().numpy()
    eGm = rel_grad_maxnorm(Gm.cpu().numpy(), G0)
    eGl = rel_grad_maxnorm(Gl.cpu().numpy(), G0)
    log(f"C4: exact {t_e*1e3:.1f} ms | monopole {t_m*1e3:.2f} ms ({t_e/t_m:.1f}x, rel G {eGm:.3e}) | "
        f"learned {t_l*1e3:.2f} ms ({t_e/t_l:.1f}x, rel G {eGl:.3e})")
    assert t_e / t_m >= 10.0
    assert eGm <= 1e-3


def test_committed_checkpoint_at_c4():
    """The committed checkpoint on the level-7 workload (327,680 faces, theta 0.5): its gate was
    chosen on held-out training-family shapes (mlp_train.select_gate), not on this workload.  The
    learned far field must be >= 10x faster than the exact kernel at <= 1e-3 gradient max-norm
    error, and no farther from the exact gradient than the plain monopole."""
    import os
    import torch
    T = tpe()
    ckpt = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2509_22110_amd", "data",
                        "farfield_mlp.bin")
    m = T.MLP.load(ckpt)
    c = M.make_config("C4")
    Xd, Fd = upload(c.X, c.F)
    tree = T.build_tree(Xd, Fd)

    def timed(fn, reps=3):
        fn(); torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out
    t_e, (E0, G0) = timed(lambda: T.gradient(Xd, Fd), reps=2)
    _, (Em, Gm) = timed(lambda: T.farfield(tree, Xd, Fd, theta=0.5))
    t_l, (El, Gl) = timed(lambda: T.farfield(tree, Xd, Fd, theta=0.5, mlp=m))
    G0 = G0.cpu().numpy()
    eGm = rel_grad_maxnorm(Gm.cpu().numpy(), G0)
    eGl = rel_grad_maxnorm(Gl.cpu().numpy(), G0)
    eEl = rel_energy(float(El.cpu()), float(E0.cpu()))
    eEm = rel_energy(float(Em.cpu()), float(E0.cpu()))
    log(f"C4 committed checkpoint (gate {m.gate():.3f}): exact {t_e*1e3:.1f} ms, learned {t_l*1e3:.2f} ms "
        f"({t_e/t_l:.1f}x), rel G {eGl:.3e} (monopole {eGm:.3e}), rel E {eEl:.3e} (monopole {eEm:.3e})")
    assert t_e / t_l >= 10.0
    assert eGl <= 1e-3 and eGl <= eGm
    assert eEl < eEm  # the gain the network brings at the same theta: energy and gradient both closer


def test_learned_against_the_monopole_at_equal_time():
    """What the committed network is worth against the method without it at the same cost: the
    monopole far field at the smaller theta that takes no longer than the learned far field at
    theta 0.5.  Measured: the monopole at theta 0.35-0.4 is as fast and 3-4x more accurate, so the
    per-face correction does not pay for its cost; the test records that ranking (a network that
    beat it would fail the last assertion, and the conclusion should then be revised)."""
    import os
    import torch
    T = tpe()
    ckpt = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2509_22110_amd", "data",
                        "farfield_mlp.bin")
    m = T.MLP.load(ckpt)
    c = M.make_config("C4")
    Xd, Fd = upload(c.X, c.F)
    _, G0 = T.gradient(Xd, Fd)
    G0 = G0.cpu().numpy()
    tree = T.build_tree(Xd, Fd)
    ctx = T.context(Xd.device)
    ctx.set_option(T.OPT_SYNC_CHECKS, 0)

    def timed(theta, mlp, reps=5):
        T.farfield(tree, Xd, Fd, theta=theta, mlp=mlp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            E, G = T.farfield(tree, Xd, Fd, theta=theta, mlp=mlp)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, rel_grad_maxnorm(G.cpu().numpy(), G0)
    try:
        t_l, e_l = timed(0.5, m)
        mono = {th: timed(th, None) for th in (0.5, 0.45, 0.4, 0.35)}
        ctx.sync_check()
    finally:
        ctx.set_option(T.OPT_SYNC_CHECKS, 1)
    log(f"learned theta 0.5: {t_l*1e3:.2f} ms, rel G {e_l:.3e}; monopole: " +
        ", ".join(f"theta {th}: {t*1e3:.2f} ms, {e:.3e}" for th, (t, e) in mono.items()))
    errs = [e for _, e in mono.values()]
    assert all(a > b for a, b in zip(errs, errs[1:]))  # smaller theta, smaller error
    within = [th for th, (t, _) in mono.items() if t <= t_l]
    assert within, "no monopole setting as fast as the learned far field"
    best = min(mono[th][1] for th in within)
    assert best < e_l  # the monopole at equal time dominates the committed per-face network


def test_c5_learned_flow_judged():
    """Level-8 workload (1,310,720 faces, gap 0.01): 100 explicit gradient-flow steps driven by
    the learned far field (committed checkpoint) on a tree built once, with the exact path as the
    judge every 10th step.  The degree-32 wrinkles hold pairs much closer than the gap, so the
    explicit step is controlled by rejection: it starts at dt = 1e-3 / max|G| (no vertex moves
    more than a tenth of the gap) and is halved until the energy decreases."""
    import os
    import torch
    from paper_2509_22110_amd.flow import RHO, ALPHA, gradient_flow_backtracking
    T = tpe()
    ckpt = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2509_22110_amd", "data",
                        "farfield_mlp.bin")
    m = T.MLP.load(ckpt)
    c = M.make_config("C5")
    Xd, Fd = upload(c.X, c.F)
    tree = T.build_tree(Xd, Fd)
    _, G0 = T.farfield(tree, Xd, Fd, theta=0.5, scale=RHO / ALPHA, mlp=m)
    dt = 1e-3 / float(G0.abs().max())
    t0 = time.time()
    rec = gradient_flow_backtracking(Xd, Fd, 100, dt, tree=tree, theta=0.5, mlp=m, judge_every=10, grow=1.25)
    torch.cuda.synchronize()
    log(f"C5 flow: dt {dt:.3e} -> {rec.dts[-1]:.3e} ({rec.rejected} rejected), {time.time() - t0:.1f} s, "
        f"E {rec.energies[0]:.6e} -> {rec.energies[-1]:.6e}, judge {[(k, float(f'{e:.3e}')) for k, e in rec.judge]}")
    assert len(rec.energies) == 100
    assert all(b < a for a, b in zip(rec.energies, rec.energies[1:]))
    assert len(rec.judge) == 10 and max(e for _, e in rec.judge) <= 1e-3
