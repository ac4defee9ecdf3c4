"""MI355X-native tangent-point energy: Python binding of libtpe (see include/tpe.h).

This module only marshals arguments: every step of the computation runs in the HIP kernels of
``libtpe.so``.  PyTorch supplies device memory and the stream.  The library must have been built
(``python -m paper_2509_22110_amd.build``); if it is missing, importing the binding's functions
raises — there is no CPU fallback.

    E = energy(X, F)                   # X: cuda float64 [V,3], F: cuda int32 [nF,3]
    E, G = gradient(X, F)              # G = dE/dX
    E = TPEFunction.apply(X, F)        # autograd: backward runs the hand-written gradient
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

__all__ = ["TPEError", "lib", "energy", "gradient", "energy_p3", "gradient_p3", "sort_pairs", "build_tree_p3", "farfield_p3", "conf_energy", "conf_gradient", "pair_count", "TPEFunction",
           "tpe_energy",
           "context", "LIB_PATH", "STATUS", "Tree", "build_tree", "farfield", "MLP"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtpe.so")

STATUS = {0: "ok", -1: "invalid argument", -2: "degenerate face", -3: "non-finite",
          -4: "out of memory", -5: "HIP error", -6: "unsupported"}

OPT_SYNC_CHECKS = 1
OPT_TARGET_WAVES = 2
OPT_KERNEL_TIMING = 3
OPT_QUADRATURE = 4
OPT_SYMMETRIC = 5
OPT_SYM_WAVES = 6
OPT_SYM_BARRIERS = 7


class TPEError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"libtpe error {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


_lib = None
_lock = threading.RLock()


def lib():
    """Load libtpe.so (after torch, so both share one HIP runtime).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2509_22110_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "tpe_version": ([], I),
            "tpe_create": ([ctypes.POINTER(P), I, P], I),
            "tpe_destroy": ([P], I),
            "tpe_set_stream": ([P, P], I),
            "tpe_set_option": ([P, I, I64], I),
            "tpe_last_error": ([P], ctypes.c_char_p),
            "tpe_check": ([P], I),
            "tpe_energy": ([P, P, I64, P, I64, D, D, D, P], I),
            "tpe_gradient": ([P, P, I64, P, I64, D, D, D, P, P], I),
            "tpe_gradient_noalloc": ([P, P, I64, P, I64, D, D, D, P, P], I),
            "tpe_energy_p3": ([P, P, I64, P, I64, D, D, D, P], I),
            "tpe_sort_pairs": ([P, P, P, I64, I], I),
            "tpe_gradient_p3": ([P, P, I64, P, I64, D, D, D, P, P], I),
            "tpe_conf_energy": ([P, P, I64, P, I64, P, I64, P, I64, D, D, D, P], I),
            "tpe_conf_gradient": ([P, P, I64, P, I64, P, I64, P, I64, D, D, D, P, P], I),
            "tpe_pair_count": ([P, P, I64, I64, ctypes.POINTER(I64)], I),
            "tpe_kernel_time": ([P, ctypes.POINTER(D), ctypes.POINTER(I64)], I),
            "tpe_exact_plan": ([P, I64, I64, ctypes.c_int32, P], I),
            "tpe_build_tree": ([P, P, I64, P, I64, ctypes.c_int32, ctypes.POINTER(P)], I),
            "tpe_tree_destroy": ([P], I),
            "tpe_tree_order": ([P, P, P, I64], I),
            "tpe_farfield": ([P, P, P, I64, P, I64, D, D, D, D, P, P, P], I),
            "tpe_farfield_dual": ([P, P, P, I64, P, I64, D, D, D, D, P, P], I),
            "tpe_build_tree_p3": ([P, P, I64, P, I64, ctypes.c_int32, ctypes.POINTER(P)], I),
            "tpe_farfield_p3": ([P, P, P, I64, P, I64, D, D, D, D, P, P, P], I),
            "tpe_farfield_stats": ([P, ctypes.POINTER(I64)], I),
            "tpe_farfield_samples": ([P, P, P, I64, P, I64, D, ctypes.c_uint64, D, ctypes.c_int32, I64, P, P, P, P],
                                     I),
            "tpe_mlp_create": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_uint64, ctypes.POINTER(P)], I),
            "tpe_mlp_destroy": ([P], I),
            "tpe_mlp_num_params": ([P], I64),
            "tpe_mlp_get_params": ([P, P, P, I64], I),
            "tpe_mlp_set_params": ([P, P, P, I64], I),
            "tpe_mlp_forward": ([P, P, P, I64, P], I),
            "tpe_mlp_set_gate": ([P, P, ctypes.c_float], I),
            "tpe_mlp_get_gate": ([P, P, ctypes.POINTER(ctypes.c_float)], I),
            "tpe_mlp_set_smoothness": ([P, P, ctypes.c_float], I),
            "tpe_mlp_train_step": ([P, P, P, P, I64, ctypes.c_float, P], I),
            "tpe_mlp_gradient": ([P, P, P, P, I64, P], I),
            "tpe_mlp_save": ([P, P, ctypes.c_char_p], I),
            "tpe_mlp_load": ([P, ctypes.c_char_p, ctypes.POINTER(P)], I),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return L


class _Ctx:
    def __init__(self, device: int):
        self.device = device
        h = ctypes.c_void_p()
        rc = lib().tpe_create(ctypes.byref(h), device, None)
        if rc:
            raise TPEError(rc, "tpe_create")
        self.h = h

    def check(self, rc: int):
        if rc:
            msg = lib().tpe_last_error(self.h)
            raise TPEError(rc, msg.decode() if msg else "")

    def bind(self, device):
        s = torch.cuda.current_stream(device)
        self.check(lib().tpe_set_stream(self.h, ctypes.c_void_p(s.cuda_stream)))
        return self

    def set_option(self, opt: int, value: int):
        self.check(lib().tpe_set_option(self.h, opt, int(value)))

    def kernel_time(self):
        """(total_ms, count) of the dominant kernel's launches recorded since the last read."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
        self.check(lib().tpe_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def exact_plan(self, nF: int, V: int, grad: bool = True):
        """(symmetric kernel: 0 no, 1 with barriers, 2 without; its waves per work-group, bytes of
        its column partial sums, scratch bytes) of an exact call on a mesh of nF faces and V
        vertices (see tpe_exact_plan)."""
        out = (ctypes.c_int64 * 4)()
        self.check(lib().tpe_exact_plan(self.h, int(nF), int(V), 1 if grad else 0, out))
        return int(out[0]), int(out[1]), int(out[2]), int(out[3])

    def farfield_stats(self):
        """(far clusters, near columns, visited nodes, target blocks, max near columns of a block,
        max far clusters of a block) of the last far-field call."""
        out = (ctypes.c_int64 * 6)()
        self.check(lib().tpe_farfield_stats(self.h, out))
        return tuple(int(v) for v in out)

    def sync_check(self):
        """Wait for the stream and raise on device-side errors (when sync checks are off)."""
        self.check(lib().tpe_check(self.h))

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.tpe_destroy(self.h)
        except Exception:
            pass


_ctxs: dict[int, _Ctx] = {}


def context(device=None) -> _Ctx:
    """Per-device library context, bound to torch's current stream on that device."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    lib()
    with _lock:
        c = _ctxs.get(idx)
        if c is None:
            c = _ctxs[idx] = _Ctx(idx)
    return c.bind(torch.device("cuda", idx))


def _check_mesh(X: torch.Tensor, F: torch.Tensor, nodes: int = 3):
    if not (isinstance(X, torch.Tensor) and isinstance(F, torch.Tensor)):
        raise TypeError("X and F must be tensors")
    if X.device.type != "cuda" or F.device != X.device:
        raise ValueError("X and F must be on the same CUDA/HIP device")
    if X.dtype != torch.float64 or X.dim() != 2 or X.shape[1] != 3:
        raise ValueError("X must be float64 [V, 3]")
    if F.dtype != torch.int32 or F.dim() != 2 or F.shape[1] != nodes:
        raise ValueError(f"F must be int32 [nF, {nodes}]")
    return X.contiguous(), F.contiguous()


def energy(X, F, q=6.0, p=12.0, scale=1.0, out=None) -> torch.Tensor:
    """E(X) as a 0-dim float64 device tensor (exact all-pairs, paper eq. (TP) discretised)."""
    X, F = _check_mesh(X, F)
    E = out if out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_energy(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0],
                             float(q), float(p), float(scale), E.data_ptr()))
    return E


def gradient(X, F, q=6.0, p=12.0, scale=1.0, out=None, energy_out=None):
    """(E, G) with G = dE/dX float64 [V, 3] (exact all-pairs)."""
    X, F = _check_mesh(X, F)
    G = out if out is not None else torch.empty_like(X)
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_gradient(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0],
                               float(q), float(p), float(scale), E.data_ptr(), G.data_ptr()))
    return E, G


def gradient_noalloc(X, F, q=6.0, p=12.0, scale=1.0, out=None, energy_out=None):
    """gradient() without any device allocation inside the library (tpe_gradient_noalloc): pass
    `out` and `energy_out` to allocate nothing at all."""
    X, F = _check_mesh(X, F)
    G = out if out is not None else torch.empty_like(X)
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_gradient_noalloc(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0],
                                       float(q), float(p), float(scale), E.data_ptr(), G.data_ptr()))
    return E, G


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, bits: int = 32):
    """Stable in-place sort of device int32 (keys, vals) by the low `bits` bits of the keys (read
    as unsigned 32-bit integers)."""
    for t in (keys, vals):
        if t.device.type != "cuda" or t.dtype != torch.int32 or t.dim() != 1 or not t.is_contiguous():
            raise ValueError("keys and vals must be contiguous 1-D int32 device tensors")
    if keys.shape != vals.shape or keys.device != vals.device:
        raise ValueError("keys and vals must have the same shape and device")
    c = context(keys.device)
    c.check(lib().tpe_sort_pairs(c.h, keys.data_ptr(), vals.data_ptr(), keys.shape[0], int(bits)))
    return keys, vals


class _Points:
    """Sets the context's quadrature rule for one call (None: leave it as it is)."""

    def __init__(self, c, points):
        self.c, self.points = c, points

    def __enter__(self):
        if self.points is not None:
            self.c.set_option(OPT_QUADRATURE, int(self.points))

    def __exit__(self, *exc):
        if self.points is not None:
            self.c.set_option(OPT_QUADRATURE, 1)


def energy_p3(X, F10, q=6.0, p=12.0, scale=1.0, out=None, points=None) -> torch.Tensor:
    """E on curved cubic elements (X: all nodes float64 [V, 3]; F10: int32 [nF, 10], corners first),
    with `points` (1, 3 or 6) quadrature points per element on both integrals (None: the
    context's TPE_OPT_QUADRATURE)."""
    X, F10 = _check_mesh(X, F10, 10)
    E = out if out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    with _Points(c, points):
        c.check(lib().tpe_energy_p3(c.h, X.data_ptr(), X.shape[0], F10.data_ptr(), F10.shape[0],
                                    float(q), float(p), float(scale), E.data_ptr()))
    return E


def gradient_p3(X, F10, q=6.0, p=12.0, scale=1.0, out=None, energy_out=None, points=None):
    """(E, dE/dX) on curved cubic elements (see energy_p3)."""
    X, F10 = _check_mesh(X, F10, 10)
    G = out if out is not None else torch.empty_like(X)
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    with _Points(c, points):
        c.check(lib().tpe_gradient_p3(c.h, X.data_ptr(), X.shape[0], F10.data_ptr(), F10.shape[0],
                                      float(q), float(p), float(scale), E.data_ptr(), G.data_ptr()))
    return E, G


def _check_pair(X, F, Y, FY):
    X, F = _check_mesh(X, F)
    Y, FY = _check_mesh(Y, FY)
    if Y.device != X.device:
        raise ValueError("both surfaces must be on the same device")
    return X, F, Y, FY


def conf_energy(X, F, Y, FY, q=6.0, p=12.0, scale=1.0, out=None) -> torch.Tensor:
    """Confinement energy of the moving surface (X, F) against the fixed surface (Y, FY) (paper
    eq. (TPConf) discretised), as a 0-dim float64 device tensor."""
    X, F, Y, FY = _check_pair(X, F, Y, FY)
    E = out if out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_conf_energy(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], Y.data_ptr(), Y.shape[0],
                                  FY.data_ptr(), FY.shape[0], float(q), float(p), float(scale), E.data_ptr()))
    return E


def conf_gradient(X, F, Y, FY, q=6.0, p=12.0, scale=1.0, out=None, energy_out=None):
    """(E_conf, dE_conf/dX float64 [V, 3]); the confining surface (Y, FY) is fixed."""
    X, F, Y, FY = _check_pair(X, F, Y, FY)
    G = out if out is not None else torch.empty_like(X)
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_conf_gradient(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], Y.data_ptr(),
                                    Y.shape[0], FY.data_ptr(), FY.shape[0], float(q), float(p), float(scale),
                                    E.data_ptr(), G.data_ptr()))
    return E, G


class Tree:
    """Cluster tree (Morton ordering of the faces, leaves of `leaf` faces); see tpe_build_tree."""

    def __init__(self, X, F, leaf: int = 32):
        X, F = _check_mesh(X, F)
        c = context(X.device)
        h = ctypes.c_void_p()
        c.check(lib().tpe_build_tree(c.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], int(leaf),
                                     ctypes.byref(h)))
        self.h, self.nF, self.V, self.leaf, self.device = h, F.shape[0], X.shape[0], leaf, X.device

    def order(self) -> torch.Tensor:
        """The tree order: item at each tree position, int32 [n] on the tree's device (the bits of
        the u32 permutation; see tpe_tree_order)."""
        n = self.nF * getattr(self, "points", 1)
        out = torch.empty(n, dtype=torch.int32, device=self.device)
        c = context(self.device)
        c.check(lib().tpe_tree_order(c.h, self.h, out.data_ptr(), n))
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.tpe_tree_destroy(self.h)
        except Exception:
            pass


def build_tree(X, F, leaf: int = 32) -> Tree:
    return Tree(X, F, leaf)


class TreeP3(Tree):
    """Cluster tree over the quadrature points of curved cubic elements; see tpe_build_tree_p3."""

    def __init__(self, X, F10, leaf: int = 32, points: int = 3):
        X, F10 = _check_mesh(X, F10, 10)
        c = context(X.device)
        h = ctypes.c_void_p()
        c.set_option(OPT_QUADRATURE, int(points))
        try:
            c.check(lib().tpe_build_tree_p3(c.h, X.data_ptr(), X.shape[0], F10.data_ptr(), F10.shape[0], int(leaf),
                                            ctypes.byref(h)))
        finally:
            c.set_option(OPT_QUADRATURE, 1)
        self.h, self.nF, self.V, self.leaf, self.device = h, F10.shape[0], X.shape[0], leaf, X.device
        self.points = int(points)


def build_tree_p3(X, F10, leaf: int = 32, points: int = 3) -> TreeP3:
    return TreeP3(X, F10, leaf, points)


def farfield_p3(tree: TreeP3, X, F10, theta=0.5, q=6.0, p=12.0, scale=1.0, mlp=None, out=None, energy_out=None,
                want_grad=True):
    """Barnes-Hut far field (E, G) on curved cubic elements, with the tree's quadrature points."""
    X, F10 = _check_mesh(X, F10, 10)
    G = (out if out is not None else torch.empty_like(X)) if want_grad else None
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_farfield_p3(c.h, tree.h, X.data_ptr(), X.shape[0], F10.data_ptr(), F10.shape[0], float(q),
                                  float(p), float(scale), float(theta), mlp.h if mlp is not None else None,
                                  E.data_ptr(), G.data_ptr() if G is not None else None))
    return E, G


def farfield(tree: Tree, X, F, theta=0.5, q=6.0, p=12.0, scale=1.0, mlp=None, out=None, energy_out=None,
             want_grad=True):
    """Barnes-Hut far-field approximation (E, G) on `tree` (G is None when want_grad is False)."""
    X, F = _check_mesh(X, F)
    G = (out if out is not None else torch.empty_like(X)) if want_grad else None
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_farfield(c.h, tree.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], float(q),
                               float(p), float(scale), float(theta), mlp.h if mlp is not None else None,
                               E.data_ptr(), G.data_ptr() if G is not None else None))
    return E, G


def farfield_dual(tree: Tree, X, F, theta=0.5, q=6.0, p=12.0, scale=1.0, out=None, energy_out=None,
                  want_grad=True):
    """Dual-tree (cluster-cluster) approximation (E, G) on `tree`: G is the exact gradient of the
    approximate energy E (see tpe_farfield_dual)."""
    X, F = _check_mesh(X, F)
    G = (out if out is not None else torch.empty_like(X)) if want_grad else None
    E = energy_out if energy_out is not None else torch.empty((), dtype=torch.float64, device=X.device)
    c = context(X.device)
    c.check(lib().tpe_farfield_dual(c.h, tree.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0], float(q),
                                    float(p), float(scale), float(theta), E.data_ptr(),
                                    G.data_ptr() if G is not None else None))
    return E, G


class MLP:
    """Learned far-field correction network (see include/tpe.h, tpe_mlp_*)."""

    def __init__(self, device=None, seed: int = 0, _handle=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        c = context(dev)
        if _handle is None:
            h = ctypes.c_void_p()
            c.check(lib().tpe_mlp_create(c.h, 32, 64, 3, 16, int(seed), ctypes.byref(h)))
            _handle = h
        self.h = _handle
        self.n_params = int(lib().tpe_mlp_num_params(self.h))

    @classmethod
    def load(cls, path: str, device=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        c = context(dev)
        h = ctypes.c_void_p()
        c.check(lib().tpe_mlp_load(c.h, path.encode(), ctypes.byref(h)))
        return cls(dev, _handle=h)

    def save(self, path: str):
        c = context(self.device)
        c.check(lib().tpe_mlp_save(c.h, self.h, path.encode()))

    def get_params(self):
        import numpy as np
        out = np.zeros(self.n_params, dtype=np.float32)
        c = context(self.device)
        c.check(lib().tpe_mlp_get_params(c.h, self.h, out.ctypes.data, self.n_params))
        return out

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        c = context(self.device)
        c.check(lib().tpe_mlp_set_params(c.h, self.h, p.ctypes.data, self.n_params))

    def set_smoothness(self, lam: float):
        """Weight of the training loss's neighbouring-row difference term (see tpe_mlp_set_smoothness)."""
        c = context(self.device)
        c.check(lib().tpe_mlp_set_smoothness(c.h, self.h, float(lam)))

    def set_gate(self, min_s: float):
        """Apply the far-field correction only to clusters with r_B / rho >= min_s."""
        c = context(self.device)
        c.check(lib().tpe_mlp_set_gate(c.h, self.h, float(min_s)))

    def gate(self) -> float:
        c = context(self.device)
        v = ctypes.c_float()
        c.check(lib().tpe_mlp_get_gate(c.h, self.h, ctypes.byref(v)))
        return float(v.value)

    def forward(self, feats):
        feats = feats.contiguous()
        assert feats.dtype == torch.float32 and feats.shape[1] == 32
        out = torch.empty(feats.shape[0], 16, dtype=torch.float32, device=feats.device)
        c = context(feats.device)
        c.check(lib().tpe_mlp_forward(c.h, self.h, feats.data_ptr(), feats.shape[0], out.data_ptr()))
        return out

    def train_step(self, feats, targets, lr: float, loss_out=None):
        feats, targets = feats.contiguous(), targets.contiguous()
        loss = loss_out if loss_out is not None else torch.empty((), dtype=torch.float32, device=feats.device)
        c = context(feats.device)
        c.check(lib().tpe_mlp_train_step(c.h, self.h, feats.data_ptr(), targets.data_ptr(), feats.shape[0],
                                         float(lr), loss.data_ptr()))
        return loss

    def gradient(self, feats, targets):
        feats, targets = feats.contiguous(), targets.contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device=feats.device)
        c = context(feats.device)
        c.check(lib().tpe_mlp_gradient(c.h, self.h, feats.data_ptr(), targets.data_ptr(), feats.shape[0],
                                       g.data_ptr()))
        return g

    def __del__(self):
        try:
            if getattr(self, "h", None) and _lib is not None:
                _lib.tpe_mlp_destroy(self.h)
        except Exception:
            pass


def farfield_samples(tree: Tree, X, F, theta=0.5, seed=0, select_prob=0.05, quota=4, max_cluster_faces=4096,
                     mlp=None):
    """(feats [rows,32], targets [rows,16]) training samples for the learned correction; rows with
    targets[:, 15] == 0 are unused.  With `mlp`, also the fused in-walk predictions [rows,16] as a
    third element.  See tpe_farfield_samples."""
    X, F = _check_mesh(X, F)
    rows = ((F.shape[0] + 63) // 64) * quota * 64
    feats = torch.empty(rows, 32, dtype=torch.float32, device=X.device)
    targets = torch.empty(rows, 16, dtype=torch.float32, device=X.device)
    pred = torch.empty(rows, 16, dtype=torch.float32, device=X.device) if mlp is not None else None
    c = context(X.device)
    c.check(lib().tpe_farfield_samples(c.h, tree.h, X.data_ptr(), X.shape[0], F.data_ptr(), F.shape[0],
                                       float(theta), int(seed), float(select_prob), int(quota),
                                       int(max_cluster_faces), mlp.h if mlp is not None else None,
                                       feats.data_ptr(), targets.data_ptr(),
                                       pred.data_ptr() if pred is not None else None))
    return (feats, targets) if mlp is None else (feats, targets, pred)


def pair_count(F, V: int) -> int:
    """Number of ordered face pairs sharing no vertex (pair interactions per evaluation)."""
    if F.device.type != "cuda" or F.dtype != torch.int32:
        raise ValueError("F must be a cuda int32 tensor")
    F = F.contiguous()
    c = context(F.device)
    n = ctypes.c_int64(0)
    c.check(lib().tpe_pair_count(c.h, F.data_ptr(), F.shape[0], int(V), ctypes.byref(n)))
    return int(n.value)


def _energy_of(X, F, q, p, scale, tree, theta, mlp, points):
    """E of the surface (F: 3 vertex ids per face, or 10 node ids per curved element)."""
    if F.shape[1] == 10:
        if tree is None:
            return energy_p3(X, F, q, p, scale, points=points)
        return farfield_p3(tree, X, F, theta, q, p, scale, mlp, want_grad=False)[0]
    if tree is None:
        return energy(X, F, q, p, scale)
    return farfield(tree, X, F, theta, q, p, scale, mlp, want_grad=False)[0]


def _gradient_of(X, F, q, p, scale, tree, theta, mlp, points, out=None, energy_out=None):
    """(E, dE/dX) of the surface, flat faces or curved elements (see _energy_of)."""
    if F.shape[1] == 10:
        if tree is None:
            return gradient_p3(X, F, q, p, scale, out=out, energy_out=energy_out, points=points)
        return farfield_p3(tree, X, F, theta, q, p, scale, mlp, out=out, energy_out=energy_out)
    if tree is None:
        return gradient(X, F, q, p, scale, out=out, energy_out=energy_out)
    return farfield(tree, X, F, theta, q, p, scale, mlp, out=out, energy_out=energy_out)


class TPEFunction(torch.autograd.Function):
    """E = TPEFunction.apply(X, F, q, p, scale, tree, theta, mlp, points).

    forward runs the energy (exact energy kernel, or the far field on `tree`); backward runs the
    hand-written gradient of the same method (tpe_gradient, or tpe_farfield which recomputes the
    cluster moments from X) and scales it by the incoming gradient.  Only X and F are saved.
    F with 10 ints per row: curved cubic elements (tpe_gradient_p3 / tpe_farfield_p3, `points`
    quadrature points per element for the exact path).

    With a tree and theta > 0 the backward is the cluster scheme's gradient (Sec. 3.2: the inner
    integrals of eq. dTP_reordered approximated per far cluster), not the derivative of the
    far-field energy that forward returns: the cluster moments and the admissibility decisions
    are not differentiated.  Both approximate the exact pair (E, dE/dX) to the far field's
    accuracy and agree at theta = 0.  Measured at theta = 0.5 on the 20,480-face sphere along three
    directions: <backward, v> is within 4e-5 (relative) of the exact directional derivative, the
    central difference of the far-field energy within 8e-3 of it."""

    @staticmethod
    def forward(ctx, X, F, q=6.0, p=12.0, scale=1.0, tree=None, theta=0.5, mlp=None, points=None):
        ctx.save_for_backward(X, F)
        ctx.params = (q, p, scale, tree, theta, mlp, points)
        return _energy_of(X.detach(), F, q, p, scale, tree, theta, mlp, points)

    @staticmethod
    def backward(ctx, gE):
        X, F = ctx.saved_tensors
        q, p, scale, tree, theta, mlp, points = ctx.params
        _, G = _gradient_of(X.detach(), F, q, p, scale, tree, theta, mlp, points)
        return G * gE, None, None, None, None, None, None, None, None


def tpe_energy(X, F, q=6.0, p=12.0, scale=1.0, tree=None, theta=0.5, mlp=None, points=None):
    """Differentiable energy (autograd through TPEFunction)."""
    return TPEFunction.apply(X, F, q, p, scale, tree, theta, mlp, points)
