"""Explicit gradient flow X <- X - dt dE/dX driven by the library's gradient.

The paper treats the tangent-point force explicitly in time (Sec. 3.2: an implicit treatment
would need a dense system).  This harness takes plain explicit Euler steps of the energy's
gradient flow, with the exact gradient or the far field, and can judge the far field every k
steps against the exact gradient.  The update itself is one in-place device axpy.  F with 10 ints
per row is a mesh of curved cubic elements (all nodes move; `points` quadrature points per
element for the exact path, the tree's points for the far field).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _gradient_of

RHO = 1e-4
ALPHA = 6.0


@dataclass
class FlowRecord:
    energies: list = field(default_factory=list)
    judge: list = field(default_factory=list)  # (step, rel grad max-norm error of the far field)
    dts: list = field(default_factory=list)    # accepted step sizes (backtracking flow)
    rejected: int = 0                          # trial steps rejected by the backtracking flow


def gradient_flow(X, F, steps: int, dt: float, scale: float = RHO / ALPHA, tree=None, theta: float = 0.5,
                  mlp=None, judge_every: int = 0, stop_on_increase: bool = True, record: FlowRecord | None = None,
                  points=None):
    """Run `steps` explicit Euler steps in place on X (float64 cuda [V,3]); returns the record.

    With `tree` the far field (optionally with `mlp`) supplies the gradient, and every
    `judge_every`-th step the exact gradient is evaluated too and the relative max-norm error is
    recorded.  Raises FloatingPointError on a non-finite energy, and on an energy increase when
    `stop_on_increase` is set (a too-large dt for an explicit scheme)."""
    rec = record if record is not None else FlowRecord()
    G = torch.empty_like(X)
    E = torch.empty((), dtype=torch.float64, device=X.device)
    prev = None
    pts = getattr(tree, "points", None) if tree is not None else points
    for k in range(steps):
        _gradient_of(X, F, 6.0, 12.0, scale, tree, theta, mlp, points, out=G, energy_out=E)
        if tree is not None:
            if judge_every and k % judge_every == 0:
                Ee, Ge = _gradient_of(X, F, 6.0, 12.0, scale, None, theta, None, pts)
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


def gradient_flow_backtracking(X, F, steps: int, dt: float, scale: float = RHO / ALPHA, tree=None,
                               theta: float = 0.5, mlp=None, judge_every: int = 0, max_halvings: int = 40,
                               grow: float = 1.0, record: FlowRecord | None = None, points=None):
    """Explicit Euler steps with step rejection: a trial X - dt G whose energy is not below the
    current one is discarded and dt halved (at most `max_halvings` times per step, then
    FloatingPointError).  An accepted step's energy and gradient serve the next step, so each
    accepted step costs one evaluation; dt is multiplied by `grow` after an accepted step.
    `energies[k]` is the energy at the start of step k; with `tree` the far field supplies E and G,
    and every `judge_every`-th step the exact gradient at the same state judges it."""
    rec = record if record is not None else FlowRecord()
    bufs = [torch.empty_like(X), torch.empty_like(X)]
    ens = [torch.empty((), dtype=torch.float64, device=X.device) for _ in range(2)]
    Xt = torch.empty_like(X)

    pts = getattr(tree, "points", None) if tree is not None else points

    def evaluate(Y, G, E):
        _gradient_of(Y, F, 6.0, 12.0, scale, tree, theta, mlp, points, out=G, energy_out=E)
        e = float(E)
        return e if e == e and abs(e) != float("inf") else float("inf")

    cur = 0
    e = evaluate(X, bufs[cur], ens[cur])
    if e == float("inf"):
        raise FloatingPointError("non-finite energy at the start")
    for k in range(steps):
        G = bufs[cur]
        if tree is not None and judge_every and k % judge_every == 0:
            _, Ge = _gradient_of(X, F, 6.0, 12.0, scale, None, theta, None, pts)
            rec.judge.append((k, float((G - Ge).abs().max() / Ge.abs().max())))
        rec.energies.append(e)
        for _ in range(max_halvings + 1):
            torch.add(X, G, alpha=-dt, out=Xt)
            try:
                et = evaluate(Xt, bufs[1 - cur], ens[1 - cur])
            except Exception:  # a trial state the library rejects (e.g. touching faces)
                et = float("inf")
            if et < e:
                break
            rec.rejected += 1
            dt *= 0.5
        else:
            raise FloatingPointError(f"no decrease within {max_halvings} halvings at step {k}")
        X.copy_(Xt)
        rec.dts.append(dt)
        cur, e = 1 - cur, et
        dt *= grow
    return rec
