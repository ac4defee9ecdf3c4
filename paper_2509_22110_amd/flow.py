"""Explicit gradient flow X <- X - dt dE/dX driven by the library's gradient.

The paper treats the tangent-point force explicitly in time (Sec. 3.2: an implicit treatment
would need a dense system).  This harness takes plain explicit Euler steps of the energy's
gradient flow, with the exact gradient or the far field, and can judge the far field every k
steps against the exact gradient.  The update itself is one in-place device axpy.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import farfield, gradient

RHO = 1e-4
ALPHA = 6.0


@dataclass
class FlowRecord:
    energies: list = field(default_factory=list)
    judge: list = field(default_factory=list)  # (step, rel grad max-norm error of the far field)


def gradient_flow(X, F, steps: int, dt: float, scale: float = RHO / ALPHA, tree=None, theta: float = 0.5,
                  mlp=None, judge_every: int = 0, stop_on_increase: bool = True, record: FlowRecord | None = None):
    """Run `steps` explicit Euler steps in place on X (float64 cuda [V,3]); returns the record.

    With `tree` the far field (optionally with `mlp`) supplies the gradient, and every
    `judge_every`-th step the exact gradient is evaluated too and the relative max-norm error is
    recorded.  Raises FloatingPointError on a non-finite energy, and on an energy increase when
    `stop_on_increase` is set (a too-large dt for an explicit scheme)."""
    rec = record if record is not None else FlowRecord()
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=X.device)
    prev = None
    for k in range(steps):
        if tree is None:
            gradient(X, F, scale=scale, out=G, energy_out=E)
        else:
            farfield(tree, X, F, theta=theta, scale=scale, mlp=mlp, out=G, energy_out=E)
            if judge_every and k % judge_every == 0:
                Ee, Ge = gradient(X, F, scale=scale)
                err = float((G - Ge).abs().max() / Ge.abs().max())
                rec.judge.append((k, err))
        e = float(E)
        if not torch.isfinite(E):
            raise FloatingPointError(f"non-finite energy at step {k}")
        if stop_on_increase and prev is not None and e > prev:
            raise FloatingPointError(f"energy increased at step {k}: {prev} -> {e}")
        rec.energies.append(e)
        prev = e
        X.add_(G, alpha=-dt)
    return rec
