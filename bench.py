"""Benchmark of the tangent-point energy + gradient hot path on one MI355X.

One step = one exact energy + gradient call (tpe_gradient: face prep, sort, exclusion map, exact
all-pairs symmetric pair kernel, FP64 merge / finalize, vertex gather) on the level-7 workload the
metric is quoted on: the icosphere of 327,680 faces deformed by spherical harmonics of degree 2..16
at amplitude 0.15 (seed 0), with the mesh already resident in HBM.  Prints ONE JSON line:
    value     = ordered non-adjacent face pairs per second of the exact energy + gradient
    roofline  = the pair kernel: 64 flop per ordered pair (the algorithmic count of the energy +
                gradient, FMA = 2) over its own launch durations, measured with HIP events on its
                stream inside the timed region, against the FP32 vector peak; executed flop per
                pair from the committed rocprofv3 counter summary (profiles/pair_kernel_C4_flops.txt)
                and HBM bytes per launch (profiles/pair_kernel_C4_traffic.txt), both null when the
                kernel's sources have changed since they were taken
    farfield  = ms per gradient on the same workload: exact all-pairs vs the cluster-tree far field
                (monopole, learned correction, dual tree) with their errors against the exact path,
                and the HBM-bound passes (merge, finalize, vertex gather) against their algorithmic
                bytes (374 per face) with the symmetric kernel's column partials as an overhead
    c2        = the same exact step on the level-5 workload (20,480 faces)
    cpu_baseline = the FP64 CPU oracle on a bounded row sample of the same workload
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-farfield] [--no-extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 work of one ordered pair of the energy + gradient (FMA = 2), the count of the
# scatter-free form: shared terms 9 (d 3, |d|^2 5, 1/|d|^2 counted as 1), forward (x = S) 28,
# reverse (y = S) 27
FLOP_PER_PAIR = 64
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 flop/clk (packed FMA)
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per face of the passes after the pair kernel: finalize ~276 (row sums,
# geometry, vertex ids, corner positions in; three FP64 corner gradients out) + gather ~98 (corner
# gradients and indices in, vertex gradient out)
FINALIZE_GATHER_BYTES_PER_FACE = 276 + 98


def sym_kernel_name(ctx, cfg):
    """The exact pair kernel the library runs for this mesh (tpe_exact_plan)."""
    sym, nw, _, _ = ctx.exact_plan(cfg.nF, cfg.V, True)
    return {2: f"pair_sym_free_kernel<true, {nw}>", 1: f"pair_sym_kernel<true, {nw}>"}.get(sym, "pair_kernel<6,true>")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C4")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-farfield", action="store_true", help="skip the far-field comparison")
    ap.add_argument("--no-c2", action="store_true", help="skip the level-5 exact step")
    ap.add_argument("--no-row-only", action="store_true", help="skip the row-only kernel comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the confinement, quadrature, exponent and curved-element timings")
    ap.add_argument("--ff-reps", type=int, default=20)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2509_22110_amd", "data", "farfield_mlp.bin"))
    return ap.parse_args()


SOURCES = {
    "pair": ("paper_2509_22110_amd/csrc/pair.hip", "paper_2509_22110_amd/csrc/common.hpp"),
    "farfield": ("paper_2509_22110_amd/csrc/tree.hip", "paper_2509_22110_amd/csrc/farfield_common.hpp",
                 "paper_2509_22110_amd/csrc/common.hpp", "paper_2509_22110_amd/csrc/mlp_infer.hpp"),
    "finalize": ("paper_2509_22110_amd/csrc/finalize.hip", "paper_2509_22110_amd/csrc/common.hpp"),
}


def source_hash(kind):
    h = hashlib.sha256()
    for rel in SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_summary(name, kind):
    """key = value pairs of a committed rocprofv3 summary under profiles/; None if there is none or if
    it was taken on other sources of the kernel than the ones built here (source_sha256)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash(kind):
        return None
    return kv


def summary_float(kv, key):
    try:
        return float(kv[key]) if kv else None
    except (KeyError, ValueError):
        return None


def exact_leg(T, M, torch, dev, name, steps, warmup):
    """`steps` timed exact energy + gradient calls after `warmup`, with the pair kernel's launches
    timed by HIP events on the context's stream inside the timed region."""
    cfg = M.make_config(name)
    X = torch.from_numpy(cfg.X).to(dev)
    F = torch.from_numpy(cfg.F).to(dev)
    P = T.pair_count(F, cfg.V)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)
    ctx = T.context(dev)
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    for _ in range(warmup):
        T.gradient(X, F, out=G, energy_out=E)
    # and at least 100 ms of warm-up work in all: the GPU's clock ramps up over the first tens of
    # milliseconds of load (a level-5 launch takes 0.39 ms cold, 0.34 ms after ~40 launches)
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.1:
        T.gradient(X, F, out=G, energy_out=E)
        torch.cuda.synchronize()
    ctx.sync_check()
    ctx.kernel_time()  # clears the record (the event pool now exists)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        T.gradient(X, F, out=G, energy_out=E)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    ctx.sync_check()
    k_avg = k_ms / max(k_n, 1)
    tflops = FLOP_PER_PAIR * P / (k_avg * 1e-3) / 1e12
    return {"cfg": cfg, "X": X, "F": F, "P": P, "G": G, "E": E, "ms_per_step": dt / steps * 1e3,
            "value": P * steps / dt, "kernel_avg_ms": k_avg, "kernel_launches": k_n, "tflops": tflops}


def row_only_leg(T, torch, dev, X, F, P, reps):
    """The same step with the row-only pair kernel (TPE_OPT_SYMMETRIC = 0), for comparison."""
    ctx = T.context(dev)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)
    ctx.set_option(T.OPT_SYMMETRIC, 0)
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    try:
        T.gradient(X, F, out=G, energy_out=E)
        ctx.kernel_time()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            T.gradient(X, F, out=G, energy_out=E)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        r_ms, r_n = ctx.kernel_time()
    finally:
        ctx.set_option(T.OPT_KERNEL_TIMING, 0)
        ctx.set_option(T.OPT_SYMMETRIC, 1)
    ctx.sync_check()
    k = r_ms / max(r_n, 1)
    return {"kernel": "pair_kernel<6,true>", "kernel_avg_ms": round(k, 4), "ms_per_step": round(ms, 4),
            "tflops": round(FLOP_PER_PAIR * P / (k * 1e-3) / 1e12, 3)}


def farfield_leg(args, T, torch, dev, ex):
    """ms per gradient on the headline workload: exact vs cluster-tree far field (+ learned, dual
    tree), and the HBM-bound passes of the exact path."""
    cfg, X, F, G0, E0 = ex["cfg"], ex["X"], ex["F"], ex["G"], ex["E"]

    def timed(fn, reps):
        # at least 100 ms of warm-up calls (the GPU's clock ramps up over the first tens of
        # milliseconds of load), then `reps` calls back to back
        torch.cuda.synchronize()
        t_w = time.perf_counter()
        while time.perf_counter() - t_w < 0.1:
            for _ in range(4):
                fn()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, out

    t_exact = ex["ms_per_step"]
    ctx = T.context(dev)
    # merge + finalize + vertex gather of the exact path, timed with HIP events
    Gs = torch.empty_like(X)
    Es = torch.empty((), dtype=torch.float64, device=dev)
    ctx.set_option(T.OPT_KERNEL_TIMING, 2)
    ctx.kernel_time()
    for _ in range(3):
        T.gradient(X, F, out=Gs, energy_out=Es)
    fg_ms, fg_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    fg_ms /= max(fg_n, 1)
    alg = FINALIZE_GATHER_BYTES_PER_FACE * cfg.nF
    _, sym_nw, cp, _ = ctx.exact_plan(cfg.nF, cfg.V, True)  # the library's own choice and sizes
    tr = read_summary(f"gather_passes_{args.config}_traffic.txt", "finalize")
    fg = {"kernels": "sym_merge_kernel + finalize_kernel<true> + vertex_gather", "bound": "hbm",
          "ms": round(fg_ms, 4), "algorithmic_bytes": alg, "bytes_per_face": FINALIZE_GATHER_BYTES_PER_FACE,
          "achieved": round(alg / (fg_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(alg / (fg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
          "overhead": {"what": "the symmetric pair kernel's column partial sums, read once by the merge",
                       "bytes": cp, "sym_waves_per_workgroup": sym_nw,
                       "with_overhead_gbs": round((alg + cp) / (fg_ms * 1e-3) / 1e9, 1)},
          "traffic": summary_float(tr, "bytes_per_call")}
    t_tree, tree = timed(lambda: T.build_tree(X, F, leaf=32), args.ff_reps)
    g0 = float(G0.abs().max())
    e0 = float(E0)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)

    def variant(mlp):
        def call():
            T.farfield(tree, X, F, theta=args.theta, mlp=mlp, out=G, energy_out=E)

        t, _ = timed(call, args.ff_reps)
        # the evaluation kernel's own time: HIP events around its launches, in a second pass
        ctx.set_option(T.OPT_KERNEL_TIMING, 1)
        call()
        ctx.kernel_time()
        for _ in range(args.ff_reps):
            call()
        k_ms, k_n = ctx.kernel_time()
        ctx.set_option(T.OPT_KERNEL_TIMING, 0)
        st = ctx.farfield_stats()
        k_ms /= max(k_n, 1)
        near = st[1] * 64 if st[3] else 0
        # pair-equivalents: exact near pairs + one pseudo-face pair per (row, far cluster), each
        # priced at the exact kernel's 64 flop
        pe = near + 64 * st[0]
        return {"ms": round(t, 3), "speedup_vs_exact": round(t_exact / t, 2),
                "rel_grad_maxnorm": float((G - G0).abs().max()) / g0,
                "rel_energy": abs(float(E) - e0) / abs(e0),
                "eval_kernel_avg_ms": round(k_ms, 4),
                "eval_tflops": round(FLOP_PER_PAIR * pe / (k_ms * 1e-3) / 1e12, 2),
                "eval_frac": round(FLOP_PER_PAIR * pe / (k_ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
                "far_clusters": st[0], "near_pairs": near}

    out = {"workload": f"{args.config}: {cfg.name} ({cfg.nF} faces, {cfg.V} vertices), seed 0",
           "faces": cfg.nF, "theta": args.theta, "leaf": 32,
           "exact_ms": round(t_exact, 3), "tree_build_ms": round(t_tree, 3),
           "finalize_gather": fg,
           "note": "errors against the exact GPU path, itself within 1e-5 of the FP64 oracle (the far "
                   "field is also checked against the FP64 oracle at its 16 worst vertices in the "
                   "tests); far-field ms per gradient exclude the tree build (an ordering that is "
                   "reused while the moments are recomputed from X on every call)",
           "monopole": variant(None), "learned": None}
    if args.mlp and os.path.exists(args.mlp):
        mlp = T.MLP.load(args.mlp, device=dev)
        out["learned"] = variant(mlp)
        out["learned"]["checkpoint"] = os.path.relpath(args.mlp, ROOT)
        out["learned"]["gate"] = round(mlp.gate(), 4)
    t, _ = timed(lambda: T.farfield_dual(tree, X, F, theta=args.theta, out=G, energy_out=E), args.ff_reps)
    st = ctx.farfield_stats()
    out["dual_tree"] = {"ms": round(t, 3), "speedup_vs_exact": round(t_exact / t, 2),
                        "rel_grad_maxnorm": float((G - G0).abs().max()) / g0,
                        "rel_energy": abs(float(E) - e0) / abs(e0),
                        "far_cluster_pairs": st[0], "exact_face_pairs": st[1]}
    ctx.sync_check()
    return out


def cpu_leg(args, cfg, P):
    """The FP64 oracle (energy + gradient, all host threads) on a bounded sample of the workload:
    consecutive blocks of rows (each row face against every column), until cpu_seconds have passed."""
    import numpy as np

    import oracle
    nth = oracle.num_threads()
    F = cfg.F
    nF = F.shape[0]
    # ordered pairs of a row: nF minus the faces sharing a vertex with it (itself included)
    v2f = [[] for _ in range(cfg.V)]
    for f, tri in enumerate(F):
        for v in tri:
            v2f[int(v)].append(f)
    rows, pairs, t = 0, 0, 0.0
    block = 1024
    while t < args.cpu_seconds and rows < nF:
        r1 = min(nF, rows + block)
        c0 = time.perf_counter()
        oracle.gradient_rows(cfg.X, F, rows, r1, nthreads=nth)
        t += time.perf_counter() - c0
        for f in range(rows, r1):
            pairs += nF - len(set(v2f[int(F[f, 0])]) | set(v2f[int(F[f, 1])]) | set(v2f[int(F[f, 2])]))
        rows = r1
    return {"value": pairs / t, "unit": "pairs/s", "cores": nth, "kind": "oracle",
            "sample": f"FP64 oracle energy+gradient on rows [0, {rows}) of {args.config} ({cfg.name}, "
                      f"{nF} faces): {pairs} ordered pairs of the workload's {P}, {t:.1f} s on {nth} threads"}


# algorithmic FP32 work of one (moving face, confining face) pair of the confinement gradient:
# d 3, |d|^2 5, 1/|d|^2 1, n_S.d 5, t 1, t^5 t^6 4, a w / s / m 3, K 2, S0 1, Sd 6, Sdd 6
FLOP_PER_CONF_PAIR = 37


def conf_leg(args, T, M, torch, dev):
    """Confinement energy + gradient (the sphere-inversion setting: the slightly flattened unit
    sphere inside the concentric sphere of radius 1.1, both level 5, 20,480 x 20,480 faces)."""
    X, F, Y, FY = M.confinement_config(5, 5)
    Xd, Fd = torch.from_numpy(X).to(dev), torch.from_numpy(F).to(dev)
    Yd, FYd = torch.from_numpy(Y).to(dev), torch.from_numpy(FY).to(dev)
    G = torch.empty_like(Xd)
    E = torch.empty((), dtype=torch.float64, device=dev)
    pairs = F.shape[0] * FY.shape[0]
    for _ in range(3):
        T.conf_gradient(Xd, Fd, Yd, FYd, out=G, energy_out=E)
    ctx = T.context(dev)
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    ctx.kernel_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        T.conf_gradient(Xd, Fd, Yd, FYd, out=G, energy_out=E)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    k_ms, k_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    ctx.sync_check()
    k_ms /= max(k_n, 1)
    return {"workload": "flattened unit sphere (level 5, 20,480 faces) in the concentric radius-1.1 sphere "
                        "(level 5, 20,480 faces)", "pairs": pairs, "ms_per_call": round(dt * 1e3, 4),
            "pairs_per_s": pairs / dt, "kernel": "pair_kernel<6,true,CONF>", "kernel_avg_ms": round(k_ms, 4),
            "kernel_tflops": round(FLOP_PER_CONF_PAIR * pairs / (k_ms * 1e-3) / 1e12, 2),
            "flop_per_pair": FLOP_PER_CONF_PAIR}


def quad_leg(args, T, M, torch, dev, cfg, X, F):
    """The exact gradient with the 6-point (degree-4) rule on both integrals: 36 point pairs per
    face pair of the same workload."""
    ctx = T.context(dev)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)
    ctx.set_option(T.OPT_QUADRATURE, 6)
    try:
        for _ in range(2):
            T.gradient(X, F, out=G, energy_out=E)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            T.gradient(X, F, out=G, energy_out=E)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    finally:
        ctx.set_option(T.OPT_QUADRATURE, 1)
    ctx.sync_check()
    pp = 36 * T.pair_count(F, cfg.V)
    return {"workload": f"{cfg.name} ({cfg.nF} faces) with 6 quadrature points per face", "point_pairs": pp,
            "ms_per_call": round(dt * 1e3, 3), "point_pairs_per_s": pp / dt}


def p3_leg(args, T, M, torch, dev, cfg, F):
    """The exact gradient on curved cubic elements of the same sphere (the level-5 icosphere's
    lattice nodes moved onto the same deformed surface; corners where the flat workload's vertices
    are), with the 6-point rule on both integrals: records, pair kernel, 10-node finalize and
    node gather."""
    X10, F10 = M.p3_sphere(5, 2, 8, 0.05, 0)
    Xd = torch.from_numpy(X10).to(dev)
    Fd = torch.from_numpy(F10).to(dev)
    ctx = T.context(dev)
    G = torch.empty_like(Xd)
    E = torch.empty((), dtype=torch.float64, device=dev)
    ctx.set_option(T.OPT_QUADRATURE, 6)
    try:
        for _ in range(2):
            T.gradient_p3(Xd, Fd, out=G, energy_out=E)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            T.gradient_p3(Xd, Fd, out=G, energy_out=E)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    finally:
        ctx.set_option(T.OPT_QUADRATURE, 1)
    ctx.sync_check()
    pp = 36 * T.pair_count(F, cfg.V)  # the elements' corners are the flat workload's faces
    return {"workload": f"{cfg.name}'s sphere as {F10.shape[0]} curved cubic elements ({X10.shape[0]} nodes), "
                        "6 quadrature points per element", "point_pairs": pp,
            "ms_per_call": round(dt * 1e3, 3), "point_pairs_per_s": pp / dt}


def p3_farfield_leg(args, T, M, torch, dev):
    """The far field on curved cubic elements: the level-6 sphere (81,920 elements, the level-5
    workload's deformation) with 3 points per element, monopole and learned, against the exact
    path with the same points."""
    X10, F10 = M.p3_sphere(6, 2, 8, 0.05, 0)
    Xd = torch.from_numpy(X10).to(dev)
    Fd = torch.from_numpy(F10).to(dev)
    ctx = T.context(dev)
    ctx.set_option(T.OPT_QUADRATURE, 3)
    try:
        E0, G0 = T.gradient_p3(Xd, Fd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E0, G0 = T.gradient_p3(Xd, Fd)
        torch.cuda.synchronize()
        t_exact = time.perf_counter() - t0
    finally:
        ctx.set_option(T.OPT_QUADRATURE, 1)
    t0 = time.perf_counter()
    tree = T.build_tree_p3(Xd, Fd, leaf=32, points=3)
    torch.cuda.synchronize()
    t_tree = time.perf_counter() - t0
    mlp = T.MLP.load(args.mlp, dev) if os.path.exists(args.mlp) else None
    out = {"workload": f"level-6 sphere as {F10.shape[0]} curved cubic elements ({X10.shape[0]} nodes), "
                       f"3 points per element, theta {args.theta}, leaf 32",
           "exact_ms": round(t_exact * 1e3, 3), "tree_build_ms": round(t_tree * 1e3, 3)}
    for name, m in (("monopole", None), ("learned", mlp)):
        if name == "learned" and m is None:
            continue
        for _ in range(2):
            E, G = T.farfield_p3(tree, Xd, Fd, theta=args.theta, mlp=m)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            E, G = T.farfield_p3(tree, Xd, Fd, theta=args.theta, mlp=m)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": round(dt * 1e3, 3), "speedup_vs_exact": round(t_exact / dt, 2),
                     "rel_grad_maxnorm": float((G - G0).abs().max() / G0.abs().max()),
                     "rel_energy": abs(float(E) - float(E0)) / abs(float(E0))}
    ctx.sync_check()
    return out


def exponents_leg(args, T, torch, dev, cfg, X, F, P):
    """The exact gradient with other exponents on the same workload: the symmetric kernel of the
    other even exponents (m = p/2 - q <= 0: -m extra multiplications by |d|^2 per pair) where the
    library takes it (barrier-free, 4 or 8 waves per work-group), else the generic row-only kernel."""
    ctx = T.context(dev)
    sym, nw, _, _ = ctx.exact_plan(cfg.nF, cfg.V, True)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)
    out = {}
    for q, p in ((4, 8), (8, 14)):
        for _ in range(2):
            T.gradient(X, F, q=float(q), p=float(p), out=G, energy_out=E)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            T.gradient(X, F, q=float(q), p=float(p), out=G, energy_out=E)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ctx.set_option(T.OPT_KERNEL_TIMING, 1)
        ctx.kernel_time()
        for _ in range(reps):
            T.gradient(X, F, q=float(q), p=float(p), out=G, energy_out=E)
        k_ms, k_n = ctx.kernel_time()
        ctx.set_option(T.OPT_KERNEL_TIMING, 0)
        ctx.sync_check()
        out[f"q{q}_p{p}"] = {"ms_per_call": round(dt * 1e3, 4), "pairs_per_s": P / dt,
                             "kernel": (f"pair_sym_free_gen_kernel<true, {nw}, {q}, {q - p // 2}>"
                                        if sym == 2 and nw in (4, 8) else f"pair_kernel<{q},true,false,true>"),
                             "kernel_avg_ms": round(k_ms / max(k_n, 1), 4)}
    return {"workload": f"{cfg.name} ({cfg.nF} faces), exact energy+gradient", "pairs": P, **out}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              f"multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2509_22110_amd as T
    from paper_2509_22110_amd import meshes as M

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = T.context(dev)
    ctx.set_option(T.OPT_SYNC_CHECKS, 0)
    if args.calib_copy_mb:
        src = torch.empty(args.calib_copy_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ex = exact_leg(T, M, torch, dev, args.config, args.steps, args.warmup)
    cfg, P = ex["cfg"], ex["P"]
    fl = read_summary(f"pair_kernel_{args.config}_flops.txt", "pair")
    tr = read_summary(f"pair_kernel_{args.config}_traffic.txt", "pair")
    exec_flop = summary_float(fl, "flop_per_launch")
    roofline = {"bound": "alu", "achieved": round(ex["tflops"], 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ex["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": summary_float(tr, "bytes_per_launch"), "kernel": sym_kernel_name(ctx, cfg),
                "kernel_avg_ms": round(ex["kernel_avg_ms"], 4), "kernel_launches": ex["kernel_launches"],
                "flop_per_pair": FLOP_PER_PAIR, "pairs_per_launch": P,
                "executed_flop_per_pair": round(exec_flop / P, 2) if exec_flop else None,
                "executed_tflops": round(exec_flop / (ex["kernel_avg_ms"] * 1e-3) / 1e12, 3) if exec_flop else None}
    if not args.no_row_only:
        roofline["row_only"] = row_only_leg(T, torch, dev, ex["X"], ex["F"], P, 3)

    ff = None if args.no_farfield else farfield_leg(args, T, torch, dev, ex)
    cpu = None if args.no_cpu else cpu_leg(args, cfg, P)
    out = {
        "metric": "TP pair interactions/s (energy+grad); ms/gradient at 327k tris vs exact FP64",
        "value": ex["value"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ex["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg.name} ({cfg.nF} faces, {cfg.V} vertices), seed 0, "
                               "exact all-pairs energy+gradient, (q,p)=(6,12)",
                   "faces": cfg.nF, "pairs": P, "q": 6, "p": 12, "parallelism": "single-gpu"},
        "roofline": roofline,
        "farfield": ff,
        "cpu_baseline": cpu,
    }
    del ex
    if not args.no_c2 and args.config != "C2":
        c2 = exact_leg(T, M, torch, dev, "C2", 200, 5)
        out["c2"] = {"workload": f"C2: {c2['cfg'].name} ({c2['cfg'].nF} faces), exact energy+gradient",
                     "pairs": c2["P"], "ms_per_step": round(c2["ms_per_step"], 4), "pairs_per_s": c2["value"],
                     "kernel": sym_kernel_name(ctx, c2["cfg"]), "kernel_avg_ms": round(c2["kernel_avg_ms"], 4),
                     "achieved": round(c2["tflops"], 3),
                     "frac": round(c2["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4)}
        if not args.no_row_only:
            out["c2"]["row_only"] = row_only_leg(T, torch, dev, c2["X"], c2["F"], c2["P"], 10)
        if not args.no_extra:
            out["confinement"] = conf_leg(args, T, M, torch, dev)
            out["quadrature6"] = quad_leg(args, T, M, torch, dev, c2["cfg"], c2["X"], c2["F"])
            out["other_exponents"] = exponents_leg(args, T, torch, dev, c2["cfg"], c2["X"], c2["F"], c2["P"])
            out["p3_elements"] = p3_leg(args, T, M, torch, dev, c2["cfg"], c2["F"])
    if not args.no_extra and not args.no_farfield:
        out["p3_farfield"] = p3_farfield_leg(args, T, M, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
