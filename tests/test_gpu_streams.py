"""Calls of one context on alternating streams (the binding binds torch's current stream on every
call) stay ordered: each call waits for the end of the previous call when that ran on another
stream, so they never share the scratch arena at the same time, and a call that grows the arena
frees the old one only after every earlier user is done.  With the synchronising checks off (no
host sync inside the calls) the results must be the bits of the same calls on one stream."""
import numpy as np
import pytest

from paper_2509_22110_amd import meshes as M
from tests.gpu_util import log, needs_gpu, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_alternating_streams_match_one_stream():
    import torch
    T = tpe()
    small = M.make_config("C1")
    X4, F4 = M.icosphere(4)
    X4 = M.sh_deform(X4, 2, 8, 0.05, 3)[0]
    big = M.make_config("C2")
    meshes = [upload(small.X, small.F), upload(X4, F4), upload(big.X, big.F)]
    trees = [T.build_tree(X, F) for X, F in meshes]

    def calls():
        # exact gradients and far fields, small -> medium -> large (the arena grows twice) -> small
        seq = []
        for k in (0, 1, 2, 0, 1):
            X, F = meshes[k]
            seq.append(("exact", k, lambda X=X, F=F: T.gradient(X, F)))
            seq.append(("far", k, lambda X=X, F=F, t=trees[k]: T.farfield(t, X, F, theta=0.5)))
        return seq

    ctx = T.context(meshes[0][0].device)
    ctx.set_option(T.OPT_SYNC_CHECKS, 0)
    try:
        # references: every call on the default stream, synchronised after each
        ref = []
        for _, _, f in calls():
            E, G = f()
            torch.cuda.synchronize()
            ref.append((float(E.cpu()), G.cpu().numpy()))
        # a fresh context whose arena starts small, then alternate two streams without host syncs
        T._ctxs.pop(meshes[0][0].device.index, None)
        ctx2 = T.context(meshes[0][0].device)
        ctx2.set_option(T.OPT_SYNC_CHECKS, 0)
        s1 = torch.cuda.Stream()
        s2 = torch.cuda.Stream()
        outs = []
        for rep in range(2):
            for i, (_, _, f) in enumerate(calls()):
                with torch.cuda.stream(s1 if (i + rep) % 2 == 0 else s2):
                    outs.append(f())
        torch.cuda.synchronize()
        ctx2.sync_check()
        bad = 0
        for i, (E, G) in enumerate(outs):
            Er, Gr = ref[i % len(ref)]
            same = float(E.cpu()) == Er and np.array_equal(G.cpu().numpy(), Gr)
            bad += not same
        log("alternating streams: calls", len(outs), "differing", bad)
        assert bad == 0
    finally:
        T.context(meshes[0][0].device).set_option(T.OPT_SYNC_CHECKS, 1)
