"""Benchmark of the exact tangent-point energy + gradient hot path on one MI355X.

One step = one tpe_gradient call (face prep, Morton sort, exclusion map, exact all-pairs pair
kernel, FP64 finalize, vertex gather) on the level-5 deformed sphere (20,480 faces, l = 2..8
spherical-harmonic deformation, a_lm ~ N(0, 0.05^2), seed 0), with the mesh already resident in
HBM.  Prints ONE JSON line:
    value     = ordered non-adjacent face pairs evaluated per second (energy + gradient)
    roofline  = the pair kernel's algorithmic FP32 rate (55 flop per ordered pair, the row
                formulation) over its own launch durations, measured with HIP events on the
                stream it runs on, vs the FP32 vector peak; the symmetric kernel that runs by
                default evaluates each unordered pair once and executes 40.5 flop per ordered pair
                (executed_tflops); traffic = HBM bytes per launch from the committed rocprofv3
                counter summary (profiles/pair_kernel_C2_traffic.txt), null when the kernel's
                sources have changed since it was taken; row_only = the same step with the row-only
                pair kernel (TPE_OPT_SYMMETRIC = 0), for comparison
    confinement = the confinement energy + gradient of a flattened sphere in a radius-1.1 sphere
                (20,480 x 20,480 faces): pairs/s and the kernel's algorithmic FP32 rate
    farfield  = ms per gradient on the level-7 workload (327,680 faces): exact all-pairs vs the
                cluster-tree far field (monopole, and with the learned correction), with their
                relative errors against the exact path
    cpu_baseline = the FP64 CPU oracle, timed on this host on the same mesh
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-farfield]
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

# algorithmic FP32 work of one ordered pair in the energy + gradient form (FMA = 2, rcp = 1):
# d 3, |d|^2 5, 1/|d|^2 1, n_S.d 5, n_T.d 5, t and tau 2, powers 8, a w / s / s' 3,
# t^6+tau^6 and m 2, K 2, S0 1, Sd 6, Sdd 6, Sn 6
FLOP_PER_PAIR = 55
# FP32 work the symmetric kernel executes per unordered pair (FMA = 2, rcp = 1), credited to both
# faces: shared d 3, |d|^2 5, rcp 1, n_S.d 5, n_T.d 5, t and tau 2, powers 6, T1 and U1 2,
# t^6+tau^6 3, w e 1 (33); the row face's 11 sums 24; the column face's 11 sums 24 (contributions of
# two rows per lane combined, then added to the rotating column sums); 81 = 40.5 per ordered pair
EXEC_FLOP_PER_PAIR_SYM = 40.5
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 flop/clk (packed FMA)
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per face of the passes after the symmetric pair kernel: the merge reads one
# row segment (8 FP32 sums = 32 B) plus the column partials (counted apart) and writes the 11 FP64
# row sums (88 B); the finalize reads them (88 B), {a, |w|, n} (40 B), vertex ids (16 B) and its
# three vertices (72 B) and writes three corner gradients (72 B); the gather reads 3 corner indices
# (12 B) and the corners (72 B) and per vertex (V ~ F/2) an offset (4 B) and writes G (24 B)
MERGE_FINALIZE_GATHER_BYTES_PER_FACE = 32 + 88 + 88 + 40 + 16 + 72 + 72 + 12 + 72 + (4 + 24) // 2
SYM_MAX_COLPART_BYTES = 64 << 30


def sym_colpart_bytes(nF, na=8):
    """Bytes of the symmetric pair kernel's column partial sums, which the finalize reads once: one
    FP32 sum per (symmetric unit, column, accumulator); super blocks of 512 faces, units of 64
    columns, the 8 chunks of a super block's own faces excluded.  0 when the library takes the
    row-only kernel (above its 6 GiB cap)."""
    fp = -(-nF // 512) * 512
    nsb, nch = fp // 512, fp // 64
    units = nsb * (nch - 8) - 8 * nsb * (nsb - 1) // 2
    b = units * na * 64 * 4
    return b if b <= SYM_MAX_COLPART_BYTES else 0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-farfield", action="store_true", help="skip the level-7 far-field comparison")
    ap.add_argument("--farfield-only", action="store_true", help="run only the level-7 far-field comparison")
    ap.add_argument("--ff-config", default="C4")
    ap.add_argument("--ff-reps", type=int, default=5)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--no-conf", action="store_true", help="skip the confinement, 6-point-quadrature and other-exponent timings")
    ap.add_argument("--mlp", default=os.path.join(ROOT, "paper_2509_22110_amd", "data", "farfield_mlp.bin"))
    return ap.parse_args()


PAIR_SOURCES = ("paper_2509_22110_amd/csrc/pair.hip", "paper_2509_22110_amd/csrc/common.hpp")


def pair_source_hash():
    h = hashlib.sha256()
    for rel in PAIR_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic():
    """HBM bytes per pair-kernel launch from the committed rocprofv3 counter summary; None if there
    is none or if it was taken on other sources of the kernel than the ones built here."""
    path = os.path.join(ROOT, "profiles", "pair_kernel_C2_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != pair_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def farfield_leg(args, T, M, torch, dev):
    """ms per gradient on the level-7 workload: exact vs cluster-tree far field (+ learned)."""
    cfg = M.make_config(args.ff_config)
    X = torch.from_numpy(cfg.X).to(dev)
    F = torch.from_numpy(cfg.F).to(dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3, out

    G0 = torch.empty_like(X)
    E0 = torch.empty((), dtype=torch.float64, device=dev)
    t_exact, _ = timed(lambda: T.gradient(X, F, out=G0, energy_out=E0), max(1, args.ff_reps // 2))
    ctx = T.context(dev)
    # the exact pair kernel at this size, timed with HIP events (the same roofline as the main line)
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    ctx.kernel_time()
    T.gradient(X, F, out=G0, energy_out=E0)
    k_ms, k_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    k_ms /= max(k_n, 1)
    pairs = T.pair_count(F, cfg.V)
    k_tflops = FLOP_PER_PAIR * pairs / (k_ms * 1e-3) / 1e12
    exact_kernel = {"kernel": "pair_sym_kernel<true>", "kernel_avg_ms": round(k_ms, 3), "pairs": pairs,
                    "achieved": round(k_tflops, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(k_tflops / FP32_VECTOR_PEAK_TFLOPS, 4)}
    # the HBM-bound passes of the exact path (finalize + vertex gather), timed with HIP events
    ctx.set_option(T.OPT_KERNEL_TIMING, 2)
    ctx.kernel_time()
    for _ in range(2):
        T.gradient(X, F, out=G0, energy_out=E0)
    fg_ms, fg_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    fg_ms /= max(fg_n, 1)
    cp_bytes = sym_colpart_bytes(cfg.nF)
    fg_bytes = MERGE_FINALIZE_GATHER_BYTES_PER_FACE * cfg.nF + cp_bytes
    fg = {"kernels": "sym_merge_kernel + finalize_kernel<true> + vertex_gather", "bound": "hbm", "ms": round(fg_ms, 4),
          "algorithmic_bytes": fg_bytes, "column_partial_bytes": cp_bytes, "achieved": round(fg_bytes / (fg_ms * 1e-3) / 1e9, 1),
          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(fg_bytes / (fg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    t_tree, tree = timed(lambda: T.build_tree(X, F, leaf=32), args.ff_reps)
    g0 = float(G0.abs().max())
    e0 = float(E0)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)

    def variant(mlp):
        t, _ = timed(lambda: T.farfield(tree, X, F, theta=args.theta, mlp=mlp, out=G, energy_out=E), args.ff_reps)
        return {"ms": round(t, 3), "speedup_vs_exact": round(t_exact / t, 2),
                "rel_grad_maxnorm": float((G - G0).abs().max()) / g0,
                "rel_energy": abs(float(E) - e0) / abs(e0)}

    out = {"workload": f"{args.ff_config}: {cfg.name} ({cfg.nF} faces, {cfg.V} vertices), seed 0",
           "faces": cfg.nF, "theta": args.theta, "leaf": 32,
           "exact_ms": round(t_exact, 3), "exact_kernel": exact_kernel, "tree_build_ms": round(t_tree, 3),
           "finalize_gather": fg,
           "note": "errors against the exact FP32/FP64 path (itself parity-tested against the FP64 "
                   "oracle); far-field ms per gradient exclude the tree build (an ordering that is "
                   "reused while the moments are recomputed from X on every call)",
           "monopole": variant(None), "learned": None}
    if args.mlp and os.path.exists(args.mlp):
        mlp = T.MLP.load(args.mlp, device=dev)
        out["learned"] = variant(mlp)
        out["learned"]["checkpoint"] = os.path.relpath(args.mlp, ROOT)
        out["learned"]["gate"] = round(mlp.gate(), 4)
    # dual tree (both integrals clustered) on the same tree
    t, _ = timed(lambda: T.farfield_dual(tree, X, F, theta=args.theta, out=G, energy_out=E), args.ff_reps)
    st = T.context(dev).farfield_stats()
    out["dual_tree"] = {"ms": round(t, 3), "speedup_vs_exact": round(t_exact / t, 2),
                        "rel_grad_maxnorm": float((G - G0).abs().max()) / g0,
                        "rel_energy": abs(float(E) - e0) / abs(e0),
                        "far_cluster_pairs": st[0], "exact_face_pairs": st[1]}
    T.context(dev).sync_check()
    return out


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
    return {"workload": f"{args.config} with 6 quadrature points per face", "point_pairs": pp,
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
    return {"workload": f"{args.config}'s sphere as {F10.shape[0]} curved cubic elements ({X10.shape[0]} nodes), "
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
    """The exact gradient with other exponents (the generic pair kernel, -m extra multiplications
    by |d|^2 per pair) on the same workload."""
    ctx = T.context(dev)
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
                             "kernel": f"pair_kernel<{q},true,false,true>",
                             "kernel_avg_ms": round(k_ms / max(k_n, 1), 4)}
    return {"workload": f"{args.config} ({cfg.nF} faces), exact energy+gradient", "pairs": P, **out}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              f"multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2509_22110_amd as T
    from paper_2509_22110_amd import meshes as M

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = M.make_config(args.config)
    X = torch.from_numpy(cfg.X).to(dev)
    F = torch.from_numpy(cfg.F).to(dev)
    P = T.pair_count(F, cfg.V)
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=dev)
    ctx = T.context(dev)
    ctx.set_option(T.OPT_SYNC_CHECKS, 0)
    if args.farfield_only:
        print(json.dumps({"farfield": farfield_leg(args, T, M, torch, dev)}), flush=True)
        return

    if args.calib_copy_mb:
        src = torch.empty(args.calib_copy_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        T.gradient(X, F, out=G, energy_out=E)
    ctx.sync_check()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T.gradient(X, F, out=G, energy_out=E)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.sync_check()
    ms_per_step = dt / args.steps * 1e3
    value = P * args.steps / dt

    # dominant kernel: the pair kernel, timed with HIP events on its own stream
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    ctx.kernel_time()
    for _ in range(args.steps):
        T.gradient(X, F, out=G, energy_out=E)
    k_ms, k_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    ctx.sync_check()
    k_avg_ms = k_ms / max(k_n, 1)
    achieved = FLOP_PER_PAIR * P / (k_avg_ms * 1e-3) / 1e12
    traffic = read_traffic()
    # the row-only kernel on the same step, for comparison
    ctx.set_option(T.OPT_SYMMETRIC, 0)
    ctx.set_option(T.OPT_KERNEL_TIMING, 1)
    for _ in range(2):
        T.gradient(X, F, out=G, energy_out=E)
    ctx.kernel_time()
    reps = max(5, min(args.steps, 20))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        T.gradient(X, F, out=G, energy_out=E)
    torch.cuda.synchronize()
    ro_ms = (time.perf_counter() - t0) / reps * 1e3
    r_ms, r_n = ctx.kernel_time()
    ctx.set_option(T.OPT_KERNEL_TIMING, 0)
    ctx.set_option(T.OPT_SYMMETRIC, 1)
    ctx.sync_check()
    r_avg_ms = r_ms / max(r_n, 1)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic, "kernel": "pair_sym_kernel<true>",
                "kernel_avg_ms": round(k_avg_ms, 4), "flop_per_pair": FLOP_PER_PAIR,
                "executed_flop_per_pair": EXEC_FLOP_PER_PAIR_SYM,
                "executed_tflops": round(EXEC_FLOP_PER_PAIR_SYM * P / (k_avg_ms * 1e-3) / 1e12, 3),
                "row_only": {"kernel": "pair_kernel<6,true>", "kernel_avg_ms": round(r_avg_ms, 4),
                             "ms_per_step": round(ro_ms, 4),
                             "tflops": round(FLOP_PER_PAIR * P / (r_avg_ms * 1e-3) / 1e12, 3)}}

    ff = None if args.no_farfield else farfield_leg(args, T, M, torch, dev)
    conf = None if args.no_conf else conf_leg(args, T, M, torch, dev)
    quad = None if args.no_conf else quad_leg(args, T, M, torch, dev, cfg, X, F)
    expo = None if args.no_conf else exponents_leg(args, T, torch, dev, cfg, X, F, P)
    p3 = None if args.no_conf or args.config != "C2" else p3_leg(args, T, M, torch, dev, cfg, F)
    p3ff = None if args.no_farfield else p3_farfield_leg(args, T, M, torch, dev)

    cpu = None
    if not args.no_cpu:
        import oracle
        nth = oracle.num_threads()
        reps, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds or reps == 0:
            c0 = time.perf_counter()
            oracle.gradient(cfg.X, cfg.F, nthreads=nth)
            t_cpu += time.perf_counter() - c0
            reps += 1
        cpu = {"value": P * reps / t_cpu, "unit": "pairs/s", "cores": nth, "kind": "oracle",
               "sample": f"FP64 oracle energy+gradient, full {args.config} mesh ({cfg.nF} faces, "
                         f"{P} pairs) x {reps}, {t_cpu:.1f} s on {nth} threads"}

    out = {
        "metric": "TP pair interactions/s (energy+grad); ms/gradient at 327k tris vs exact FP64",
        "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg.name} ({cfg.nF} faces, {cfg.V} vertices), seed 0, "
                               "exact all-pairs energy+gradient, (q,p)=(6,12)",
                   "faces": cfg.nF, "pairs": P, "q": 6, "p": 12, "parallelism": "single-gpu"},
        "roofline": roofline,
        "farfield": ff,
        "confinement": conf,
        "quadrature6": quad,
        "other_exponents": expo,
        "p3_elements": p3,
        "p3_farfield": p3ff,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
