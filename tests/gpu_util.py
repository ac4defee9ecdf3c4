"""Helpers shared by the GPU tests: device availability, mesh upload, error metrics."""
import os
import sys

import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2509_22110_amd", "libtpe.so")

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")


def tpe():
    """The HIP binding; fails loudly (no fallback) when the library is missing on a machine with a GPU."""
    if not os.path.exists(LIB):
        raise RuntimeError("libtpe.so is not built; run python -m paper_2509_22110_amd.build")
    import paper_2509_22110_amd as m
    m.lib()
    return m


def upload(X, F):
    return (torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(F, dtype=np.int32)).cuda())


def rel_energy(E, Eref):
    return abs(E - Eref) / abs(Eref)


def rel_grad_maxnorm(G, Gref):
    """max |G - G*| / max |G*| over all vertex components."""
    return float(np.abs(G - Gref).max() / np.abs(Gref).max())


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()
