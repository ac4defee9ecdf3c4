"""Train the learned far-field correction on exact cluster interactions.

Training shapes are seeded level-5 and level-6 deformed spheres (seeds 1000..1199 by default;
evaluation workloads use seed 0): real spherical-harmonic deformations of random degree and
amplitude, some with an inward bump that brings two sheets together.  For every shape the
library's tree walk emits samples (features of a (face, far cluster) pair and the exact-minus-
monopole correction of the face's row sums, see tpe_farfield_samples); the network is then trained
with the library's BF16-MFMA forward/backward and Adam kernels.

    python -m paper_2509_22110_amd.mlp_train --out paper_2509_22110_amd/data/farfield_mlp.bin
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np
import torch

from . import MLP, build_tree, farfield_samples
from . import meshes as M

NOUT = 7  # used outputs: K, Sd (3), C (3)
DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "farfield_mlp.bin")


def training_shape(seed: int):
    """A seeded level-5 or level-6 deformed sphere (never seed 0, the evaluation seed)."""
    rng = np.random.default_rng(seed)
    level = 6 if seed % 4 == 0 else 5
    X, F = M.icosphere(level)
    lmax = int(rng.choice([8, 12, 16]))
    amp = float(rng.uniform(0.05, 0.2))
    X, _ = M.sh_deform_amplitude(X, 2, lmax, amp, seed)
    if seed % 3 == 0:
        X, _, _ = M.bump(X, int(rng.integers(0, X.shape[0])), float(rng.uniform(0.2, 0.4)),
                         depth=float(rng.uniform(0.3, 1.2)))
    return X, F


def collect(seeds, theta=0.5, select_prob=0.02, quota=16, max_cluster_faces=1 << 20, device="cuda", log=print):
    feats, targs = [], []
    for s in seeds:
        X, F = training_shape(s)
        Xd = torch.from_numpy(X).to(device)
        Fd = torch.from_numpy(F).to(device)
        tree = build_tree(Xd, Fd, leaf=32)
        f, t = farfield_samples(tree, Xd, Fd, theta=theta, seed=s, select_prob=select_prob, quota=quota,
                                max_cluster_faces=max_cluster_faces)
        keep = t[:, 15] > 0
        feats.append(f[keep])
        targs.append(t[keep])
    return torch.cat(feats), torch.cat(targs)


def zero_loss(T):
    w = T[:, 15]
    return float((w[:, None] * T[:, :NOUT] ** 2).sum() / (NOUT * w.sum()))


def evaluate(mlp, X, T, batch=65536):
    tot, wsum = 0.0, 0.0
    for i in range(0, X.shape[0], batch):
        y = mlp.forward(X[i:i + batch])
        t = T[i:i + batch]
        w = t[:, 15]
        tot += float((w[:, None] * (y[:, :NOUT] - t[:, :NOUT]) ** 2).sum())
        wsum += float(w.sum())
    return tot / (NOUT * wsum)


def train(mlp, X, T, epochs=8, batch=8192, lr=2e-3, seed=0, log=print, Xv=None, Tv=None):
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps = epochs * max(1, n // batch)
    step = 0
    loss = torch.empty((), dtype=torch.float32, device=X.device)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
            mlp.train_step(X[idx], T[idx], cur, loss_out=loss)
            step += 1
        msg = f"epoch {ep}: train loss {float(loss):.4e}"
        if Xv is not None:
            msg += f", val loss {evaluate(mlp, Xv, Tv):.4e} (zero-prediction {zero_loss(Tv):.4e})"
        log(msg)
    return mlp


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--shapes", type=int, default=200)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--theta", type=float, default=0.5)
    args = ap.parse_args(argv)

    def log(*a):
        print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)

    seeds = list(range(args.first_seed, args.first_seed + args.shapes))
    nval = max(1, args.shapes // 10)
    t0 = time.time()
    X, T = collect(seeds[:-nval], theta=args.theta, log=log)
    Xv, Tv = collect(seeds[-nval:], theta=args.theta, log=log)
    log(f"samples: train {X.shape[0]}, val {Xv.shape[0]} ({time.time() - t0:.1f} s)")
    mlp = MLP(seed=args.first_seed)
    train(mlp, X, T, epochs=args.epochs, log=log, Xv=Xv, Tv=Tv)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    mlp.save(args.out)
    log(f"saved {args.out}; val loss {evaluate(mlp, Xv, Tv):.4e} vs zero-prediction {zero_loss(Tv):.4e}")


if __name__ == "__main__":
    sys.exit(main())
