"""Benchmark of the exact tangent-point energy + gradient hot path on one MI355X.

One step = one tpe_gradient call (face prep, Morton sort, exclusion map, exact all-pairs pair
kernel, FP64 finalize, vertex gather) on the level-5 deformed sphere (20,480 faces, l = 2..8
spherical-harmonic deformation, a_lm ~ N(0, 0.05^2), seed 0), with the mesh already resident in
HBM.  Prints ONE JSON line:
    value     = ordered non-adjacent face pairs evaluated per second (energy + gradient)
    roofline  = the pair kernel's algorithmic FP32 rate (55 flop per pair) over its own launch
                durations, measured with HIP events on the stream it runs on, vs the FP32
                vector peak; traffic from rocprofv3 counters (see profiles/) when available
    cpu_baseline = the FP64 CPU oracle, timed on this host on the same mesh
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
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
FP32_VECTOR_PEAK_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 flop/clk (packed FMA)
HBM_PEAK_GBS = 8000.0


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
    return ap.parse_args()


def read_traffic():
    """HBM bytes per pair-kernel launch from the committed rocprofv3 counter summary, if any."""
    path = os.path.join(ROOT, "profiles", "pair_kernel_C2_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            return json.load(f).get("bytes_per_launch")
    except Exception:
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
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
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic, "kernel": "pair_kernel<6,true>",
                "kernel_avg_ms": round(k_avg_ms, 4), "flop_per_pair": FLOP_PER_PAIR}

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
