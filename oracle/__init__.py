"""FP64 CPU oracle for the tangent-point energy and its gradient.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py``.  The library's product path never imports, links or calls anything here.

The arithmetic lives in ``tpe_oracle.c`` (plain C, FP64, OpenMP over rows); this module builds it with
gcc and calls it through ctypes on NumPy arrays.  See ``tpe_oracle.c`` for the definition it follows
(paper Sec. 2.2.2, eq. (TP), one-point centroid quadrature on flat triangles, ordered pairs of faces that
share no vertex) and for the gradient's chain rule.

Also the confinement energy (paper Sec. 2.2.3, eq. (TPConf)) of a moving surface against a fixed one
(``conf_energy``, ``conf_gradient``; see ``tpe_oracle.c``).

Parity pins: closed forms (two-triangle example, sphere limit, concentric-sphere limit of the
confinement energy), exact identities (scaling law, Euler identity, zero net force and torque,
rigid-motion, orientation and permutation invariance), brute-force pair counts and central finite
differences -- see tests/test_oracle.py and tests/test_oracle_conf.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpe_oracle.c")
_SRC_FF = os.path.join(_HERE, "tpe_oracle_ff.c")
_LIB = os.path.join(_HERE, "libtpe_oracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "degenerate face", -3: "non-finite"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FP contraction)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_FF))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", _SRC, _SRC_FF, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out_path: str) -> str:
    """Compile ``sanitize_driver.c`` with both oracle sources under AddressSanitizer and
    UndefinedBehaviorSanitizer (every report fatal, the runtime linked statically) into the
    executable `out_path`: a check of the oracle's own memory accesses and arithmetic, run by the
    CPU tests."""
    subprocess.check_call([
        "gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
        "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
        "-static-libasan", _SRC, _SRC_FF, os.path.join(_HERE, "sanitize_driver.c"), "-o", out_path, "-lm",
    ])
    return out_path


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        D, I64, I32, P = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        lib.tpeo_energy.argtypes = [P, I64, P, I64, D, D, D, I32, P]
        lib.tpeo_energy_rows.argtypes = [P, I64, P, I64, D, D, D, I64, I64, I32, P]
        lib.tpeo_gradient.argtypes = [P, I64, P, I64, D, D, D, I32, P, P]
        lib.tpeo_gradient_at.argtypes = [P, I64, P, I64, D, D, D, P, I64, I32, P]
        lib.tpeo_gradient_rows.argtypes = [P, I64, P, I64, D, D, D, I64, I64, I32, P, P]
        lib.tpeo_gradient_rows.restype = I32
        lib.tpeo_conf_energy.argtypes = [P, I64, P, I64, P, I64, P, I64, D, D, D, I32, P]
        lib.tpeo_conf_gradient.argtypes = [P, I64, P, I64, P, I64, P, I64, D, D, D, I32, P, P]
        lib.tpeo_conf_energy.restype = I32
        lib.tpeo_conf_gradient.restype = I32
        lib.tpeo_gradient_quad.argtypes = [P, I64, P, I64, D, D, D, I32, I32, P, P]
        lib.tpeo_gradient_quad.restype = I32
        lib.tpeo_quad_rule.argtypes = [I32, P, P]
        lib.tpeo_quad_rule.restype = I32
        lib.tpeo_gradient_p3.argtypes = [P, I64, P, I64, D, D, D, I32, I32, P, P]
        lib.tpeo_gradient_p3.restype = I32
        lib.tpeo_p3_map.argtypes = [P, D, D, P, P, P]
        lib.tpeo_p3_map.restype = I32
        lib.tpeo_pair_count.argtypes = [P, I64]
        lib.tpeo_pair_count.restype = I64
        lib.tpeo_num_threads.argtypes = [I32]
        lib.tpeo_kd_order.argtypes = [P, I64, P, I64, I32, P]
        lib.tpeo_kd_order.restype = I32
        lib.tpeo_farfield.argtypes = [P, I64, P, I64, P, I32, D, D, D, D, I32, P, P, P]
        lib.tpeo_farfield.restype = I32
        lib.tpeo_farfield_coverage.argtypes = [P, I64, P, I64, P, I32, D, P]
        lib.tpeo_farfield_coverage.restype = I32
        lib.tpeo_sample_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        lib.tpeo_sample_hash.restype = ctypes.c_uint32
        lib.tpeo_farfield_samples.argtypes = [P, I64, P, I64, P, I32, D, ctypes.c_uint64, D, I64, I64, P, P, P, P]
        lib.tpeo_farfield_samples.restype = I64
        lib.tpeo_farfield_dual.argtypes = [P, I64, P, I64, P, I32, D, D, D, D, P, I64, I32, P, P, P]
        lib.tpeo_farfield_dual.restype = I32
        lib.tpeo_kd_order_p3.argtypes = [P, I64, P, I64, P, I32, I32, P]
        lib.tpeo_kd_order_p3.restype = I32
        lib.tpeo_farfield_p3.argtypes = [P, I64, P, I64, P, P, I32, P, I32, D, D, D, D, I32, P, P, P]
        lib.tpeo_farfield_p3.restype = I32
        lib.tpeo_farfield_coverage_p3.argtypes = [P, I64, P, I64, P, P, I32, P, I32, D, P]
        lib.tpeo_farfield_coverage_p3.restype = I32
        for f in (lib.tpeo_energy, lib.tpeo_energy_rows, lib.tpeo_gradient, lib.tpeo_gradient_at):
            f.restype = I32
        _lib = lib
    return _lib


def _prep(X, F):
    X = np.ascontiguousarray(X, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    assert X.ndim == 2 and X.shape[1] == 3 and F.ndim == 2 and F.shape[1] == 3
    return X, F


def num_threads(nthreads: int = 0) -> int:
    return int(_load().tpeo_num_threads(nthreads))


def energy(X, F, q=6.0, p=12.0, scale=1.0, nthreads=0) -> float:
    X, F = _prep(X, F)
    E = np.zeros(1)
    rc = _load().tpeo_energy(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale,
                             nthreads, E.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0])


def energy_rows(X, F, r0, r1, q=6.0, p=12.0, scale=1.0, nthreads=0) -> float:
    """Sum over rows S in [r0, r1) of a_S sum_T a_T k(S,T) (times scale)."""
    X, F = _prep(X, F)
    E = np.zeros(1)
    rc = _load().tpeo_energy_rows(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale,
                                  r0, r1, nthreads, E.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0])


def gradient(X, F, q=6.0, p=12.0, scale=1.0, nthreads=0):
    """Returns (E, G) with G = dE/dX, shape [V, 3]."""
    X, F = _prep(X, F)
    E = np.zeros(1)
    G = np.zeros_like(X)
    rc = _load().tpeo_gradient(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale,
                               nthreads, E.ctypes.data, G.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G


def gradient_rows(X, F, r0, r1, q=6.0, p=12.0, scale=1.0, nthreads=0):
    """(E_rows, G_rows): the contributions of the ordered pairs whose first face lies in [r0, r1)
    to the energy and to dE/dX (the full ones for [0, nF))."""
    X, F = _prep(X, F)
    E = np.zeros(1)
    G = np.zeros_like(X)
    rc = _load().tpeo_gradient_rows(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale,
                                    int(r0), int(r1), nthreads, E.ctypes.data, G.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G


def gradient_at(X, F, verts, q=6.0, p=12.0, scale=1.0, nthreads=0):
    """Exact dE/dx_v for the listed vertices only, shape [len(verts), 3]."""
    X, F = _prep(X, F)
    verts = np.ascontiguousarray(verts, dtype=np.int32)
    G = np.zeros((verts.size, 3))
    rc = _load().tpeo_gradient_at(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale,
                                  verts.ctypes.data, verts.size, nthreads, G.ctypes.data)
    if rc:
        raise OracleError(rc)
    return G


def pair_count(F) -> int:
    F = np.ascontiguousarray(F, dtype=np.int32)
    return int(_load().tpeo_pair_count(F.ctypes.data, F.shape[0]))


def conf_energy(X, F, Y, FY, q=6.0, p=12.0, scale=1.0, nthreads=0) -> float:
    """Confinement energy of the moving surface (X, F) against the fixed surface (Y, FY)."""
    X, F = _prep(X, F)
    Y, FY = _prep(Y, FY)
    E = np.zeros(1)
    rc = _load().tpeo_conf_energy(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], Y.ctypes.data, Y.shape[0],
                                  FY.ctypes.data, FY.shape[0], q, p, scale, nthreads, E.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0])


def conf_gradient(X, F, Y, FY, q=6.0, p=12.0, scale=1.0, nthreads=0):
    """(E_conf, dE_conf/dX [V, 3]); the confining surface is fixed."""
    X, F = _prep(X, F)
    Y, FY = _prep(Y, FY)
    E = np.zeros(1)
    G = np.zeros_like(X)
    rc = _load().tpeo_conf_gradient(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], Y.ctypes.data,
                                    Y.shape[0], FY.ctypes.data, FY.shape[0], q, p, scale, nthreads, E.ctypes.data,
                                    G.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G


def quad_rule(rule):
    """(barycentric points [Q, 3], weights [Q]) of the oracle's triangle rule (1, 3 or 6 points)."""
    b = np.zeros((6, 3))
    w = np.zeros(6)
    n = _load().tpeo_quad_rule(int(rule), b.ctypes.data, w.ctypes.data)
    if n == 0:
        raise OracleError(-1)
    return b[:n].copy(), w[:n].copy()


def gradient_quad(X, F, rule, q=6.0, p=12.0, scale=1.0, nthreads=0, want_grad=True):
    """(E_Q, dE_Q/dX) with `rule`-point quadrature on every face (G is None if not want_grad)."""
    X, F = _prep(X, F)
    E = np.zeros(1)
    G = np.zeros_like(X) if want_grad else None
    rc = _load().tpeo_gradient_quad(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], q, p, scale, int(rule),
                                    nthreads, E.ctypes.data, G.ctypes.data if want_grad else None)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G


def _prep10(X, F10):
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    F10 = np.ascontiguousarray(np.asarray(F10, dtype=np.int32))
    if X.ndim != 2 or X.shape[1] != 3 or F10.ndim != 2 or F10.shape[1] != 10:
        raise ValueError("expected X [V, 3] and F10 [nF, 10]")
    return X, F10


def p3_map(P, s, t):
    """(x, x_s, x_t) of the cubic element with nodes P [10, 3] at reference point (s, t)."""
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(10, 3))
    x, xs, xt = np.zeros(3), np.zeros(3), np.zeros(3)
    _load().tpeo_p3_map(P.ctypes.data, float(s), float(t), x.ctypes.data, xs.ctypes.data, xt.ctypes.data)
    return x, xs, xt


def gradient_p3(X, F10, rule, q=6.0, p=12.0, scale=1.0, nthreads=0, want_grad=True):
    """(E, dE/dX) on curved cubic elements (X: all nodes [V, 3]; F10: [nF, 10] node ids, corners
    first) with the `rule`-point quadrature on both integrals (G is None if not want_grad)."""
    X, F10 = _prep10(X, F10)
    E = np.zeros(1)
    G = np.zeros_like(X) if want_grad else None
    rc = _load().tpeo_gradient_p3(X.ctypes.data, X.shape[0], F10.ctypes.data, F10.shape[0], q, p, scale, int(rule),
                                  nthreads, E.ctypes.data, G.ctypes.data if want_grad else None)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G


# ---- cluster approximations (tpe_oracle_ff.c; paper Sec. 3.2) -----------------------------------------


def kd_order(X, F, leaf=32):
    """Tree order of the faces (position -> face id, uint32 [nF]): the k-d ordering of the cluster
    tree with leaves of `leaf` faces (see tpe_oracle_ff.c)."""
    X, F = _prep(X, F)
    perm = np.zeros(F.shape[0], dtype=np.uint32)
    rc = _load().tpeo_kd_order(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], int(leaf), perm.ctypes.data)
    if rc:
        raise OracleError(rc)
    return perm


def _perm(X, F, perm, leaf):
    if perm is None:
        perm = kd_order(X, F, leaf)
    return np.ascontiguousarray(perm, dtype=np.uint32)


def farfield(X, F, theta, leaf=32, perm=None, q=6.0, p=12.0, scale=1.0, nthreads=0, want_grad=True):
    """(E, G, stats) of the Barnes-Hut clustering of the inner integrals of eq. (dTP_reordered) on
    the tree `perm` (default: kd_order(X, F, leaf)); stats = (far clusters, near columns, visited
    nodes, target blocks, max near columns of a block, max far clusters of a block)."""
    X, F = _prep(X, F)
    perm = _perm(X, F, perm, leaf)
    E = np.zeros(1)
    G = np.zeros_like(X) if want_grad else None
    st = np.zeros(6, dtype=np.int64)
    rc = _load().tpeo_farfield(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], perm.ctypes.data, int(leaf),
                               float(theta), q, p, scale, nthreads, E.ctypes.data,
                               G.ctypes.data if want_grad else None, st.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G, tuple(int(v) for v in st)


def _rule(rule):
    b, w = quad_rule(rule)
    return np.ascontiguousarray(b, dtype=np.float64), np.ascontiguousarray(w, dtype=np.float64)


def kd_order_p3(X, F10, rule, leaf=32):
    """Tree order of the quadrature records of curved elements (record r = rule e + k: point k of
    element e; position -> record, uint32 [nF rule]), the k-d ordering of their positions."""
    X, F10 = _prep10(X, F10)
    b, _ = _rule(rule)
    perm = np.zeros(F10.shape[0] * len(b), dtype=np.uint32)
    rc = _load().tpeo_kd_order_p3(X.ctypes.data, X.shape[0], F10.ctypes.data, F10.shape[0], b.ctypes.data, len(b),
                                  int(leaf), perm.ctypes.data)
    if rc:
        raise OracleError(rc)
    return perm


def farfield_p3(X, F10, theta, rule, leaf=32, perm=None, q=6.0, p=12.0, scale=1.0, nthreads=0, want_grad=True):
    """(E, G, stats) of the clustering of the inner integrals on curved cubic elements, over the
    records of the `rule`-point quadrature (see tpe_oracle_ff.c); stats as for farfield."""
    X, F10 = _prep10(X, F10)
    b, w = _rule(rule)
    if perm is None:
        perm = kd_order_p3(X, F10, rule, leaf)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    E = np.zeros(1)
    G = np.zeros_like(X) if want_grad else None
    st = np.zeros(6, dtype=np.int64)
    rc = _load().tpeo_farfield_p3(X.ctypes.data, X.shape[0], F10.ctypes.data, F10.shape[0], b.ctypes.data,
                                  w.ctypes.data, len(b), perm.ctypes.data, int(leaf), float(theta), q, p, scale,
                                  nthreads, E.ctypes.data, G.ctypes.data if want_grad else None, st.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G, tuple(int(v) for v in st)


def farfield_coverage_p3(X, F10, theta, rule, leaf=32, perm=None):
    """farfield_coverage on the records of curved elements."""
    X, F10 = _prep10(X, F10)
    b, w = _rule(rule)
    if perm is None:
        perm = kd_order_p3(X, F10, rule, leaf)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    out = np.zeros(2, dtype=np.int64)
    rc = _load().tpeo_farfield_coverage_p3(X.ctypes.data, X.shape[0], F10.ctypes.data, F10.shape[0], b.ctypes.data,
                                           w.ctypes.data, len(b), perm.ctypes.data, int(leaf), float(theta),
                                           out.ctypes.data)
    if rc:
        raise OracleError(rc)
    return int(out[0]), int(out[1])


def farfield_coverage(X, F, theta, leaf=32, perm=None):
    """Invariants of the walk: (blocks whose faces do not see every face exactly once, far clusters
    holding a face that shares a vertex with a face of the target block)."""
    X, F = _prep(X, F)
    perm = _perm(X, F, perm, leaf)
    out = np.zeros(2, dtype=np.int64)
    rc = _load().tpeo_farfield_coverage(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], perm.ctypes.data,
                                        int(leaf), float(theta), out.ctypes.data)
    if rc:
        raise OracleError(rc)
    return int(out[0]), int(out[1])


def sample_hash(seed, block, node):
    return int(_load().tpeo_sample_hash(int(seed) & (2**64 - 1), int(block), int(node)))


def farfield_samples(X, F, theta, seed, select_prob, max_faces, leaf=32, perm=None, cap=None):
    """Learned-correction samples of the walk: dict with 'block', 'node' [n], 'feats' [n, 64, 19] and
    'targets' [n, 64, 8] (7 targets and the row weight) for every selected (block, far cluster)."""
    X, F = _prep(X, F)
    perm = _perm(X, F, perm, leaf)
    lib = _load()
    args = (X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], perm.ctypes.data, int(leaf), float(theta),
            int(seed) & (2**64 - 1), float(select_prob), int(max_faces))
    if cap is None:
        n = lib.tpeo_farfield_samples(*args, 0, None, None, None, None)
        if n < 0:
            raise OracleError(int(n))
        cap = int(n)
    blk = np.zeros(max(cap, 1), dtype=np.int32)
    node = np.zeros(max(cap, 1), dtype=np.int32)
    feats = np.zeros((max(cap, 1), 64, 19))
    targ = np.zeros((max(cap, 1), 64, 8))
    n = lib.tpeo_farfield_samples(*args, cap, blk.ctypes.data, node.ctypes.data, feats.ctypes.data,
                                  targ.ctypes.data)
    if n < 0:
        raise OracleError(int(n))
    n = min(int(n), cap)
    return {"block": blk[:n], "node": node[:n], "feats": feats[:n], "targets": targ[:n]}


def farfield_dual(X, F, theta, leaf=32, perm=None, verts=None, q=6.0, p=12.0, scale=1.0, nthreads=0,
                  want_grad=True):
    """(E, G, stats) of the dual-tree clustering: E its approximate energy, G [V or len(verts), 3] the
    exact derivative of E (complex step, lists fixed), stats = (far cluster pairs, face pairs of near
    dual leaves)."""
    X, F = _prep(X, F)
    perm = _perm(X, F, perm, leaf)
    vv = None if verts is None else np.ascontiguousarray(verts, dtype=np.int32)
    nv = X.shape[0] if vv is None else vv.size
    E = np.zeros(1)
    G = np.zeros((nv, 3)) if want_grad else None
    st = np.zeros(2, dtype=np.int64)
    rc = _load().tpeo_farfield_dual(X.ctypes.data, X.shape[0], F.ctypes.data, F.shape[0], perm.ctypes.data,
                                    int(leaf), float(theta), q, p, scale, None if vv is None else vv.ctypes.data,
                                    nv, nthreads, E.ctypes.data, G.ctypes.data if want_grad else None,
                                    st.ctypes.data)
    if rc:
        raise OracleError(rc)
    return float(E[0]), G, tuple(int(v) for v in st)
