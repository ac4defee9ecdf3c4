"""tpe_gradient_noalloc (the entry point that allocates nothing) through the C ABI, against
tpe_gradient: bit-identical to the row-only path (TPE_OPT_SYMMETRIC = 0) and within the parity
bounds (energy 1e-6, gradient max-norm 1e-5 relative) of the default symmetric path, on two calls
in a row, the second on a smaller mesh (the shared scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest

from paper_2509_22110_amd import meshes as M
from tests.gpu_util import log, needs_gpu, rel_energy, rel_grad_maxnorm, tpe, upload

pytestmark = [pytest.mark.gpu, needs_gpu]


def _noalloc(T, X, F, E, G):
    c = T.context(X.device)
    rc = T.lib().tpe_gradient_noalloc(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], 6.0, 12.0, 1.0,
                                      E.data_ptr(), G.data_ptr())
    return rc, c


def test_noalloc_matches_tpe_gradient_twice():
    import torch
    T = tpe()
    big, small = M.make_config("C2"), M.make_config("C1")
    # warm-up: the HIP runtime backs the kernels' register spills (private segment) on their first
    # launch in the process; that is the runtime's per-lane scratch, not a buffer of the library
    X, F = upload(small.X, small.F)
    E = torch.empty((), dtype=torch.float64, device=X.device)
    G = torch.empty_like(X)
    rc, c = _noalloc(T, X, F, E, G)
    c.check(rc)
    results = []
    for cfg in (big, small):
        log("noalloc", cfg.name, "faces", cfg.F.shape[0])
        X, F = upload(cfg.X, cfg.F)
        E = torch.empty((), dtype=torch.float64, device=X.device)
        G = torch.empty_like(X)
        T.context(X.device)  # the context (and the library's code object) exist before the measurement
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        rc, c = _noalloc(T, X, F, E, G)
        c.check(rc)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        results.append((cfg, X, F, float(E.cpu()), G.cpu().numpy(), free0 - free1))
    for cfg, X, F, En, Gn, used in results:
        c = T.context(X.device)
        c.set_option(T.OPT_SYMMETRIC, 0)
        try:
            Er, Gr = T.gradient(X, F)
        finally:
            c.set_option(T.OPT_SYMMETRIC, 1)
        Es, Gs = T.gradient(X, F)
        eE, eG = rel_energy(En, float(Es.cpu())), rel_grad_maxnorm(Gn, Gs.cpu().numpy())
        log("  ", cfg.name, "device bytes taken by the call", used, "vs symmetric path: rel E", eE, "rel G", eG)
        assert En == float(Er.cpu()) and np.array_equal(Gn, Gr.cpu().numpy())
        assert eE <= 1e-6 and eG <= 1e-5
        assert used < (1 << 20)  # no device allocation inside the call


def test_noalloc_rejects_meshes_beyond_its_scratch():
    import torch
    T = tpe()
    c = M.make_config("C4")
    X, F = upload(c.X, c.F)
    E = torch.empty((), dtype=torch.float64, device=X.device)
    G = torch.empty_like(X)
    rc, ctx = _noalloc(T, X, F, E, G)
    msg = T.lib().tpe_last_error(ctx.h).decode()
    log("noalloc at 327,680 faces:", rc, msg)
    assert rc == -1 and "no-allocation scratch" in msg
