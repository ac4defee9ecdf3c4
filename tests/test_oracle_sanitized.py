"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every C entry point runs once on
small meshes (flat level-3 surface with a dent, its confinement, curved cubic elements -- also
their far field's tree order, walk and coverage) in a
sanitized build, which must finish without a report, and its results must be those of the regular
build (the same code; only the OpenMP split of the sums may differ)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2509_22110_amd import meshes as M


def _write(path, X, F):
    X = np.ascontiguousarray(X, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    with open(path, "wb") as f:
        f.write(np.array([X.shape[0], F.shape[0]], dtype=np.int64).tobytes())
        f.write(X.tobytes())
        f.write(F.tobytes())


def _regular(X, F, Y, FY, X10, F10):
    """The driver's lines, computed through the regular build."""
    out = {}
    E = oracle.energy(X, F, nthreads=2)
    out["energy"] = [0, E]
    E, G = oracle.gradient(X, F, nthreads=2)
    out["gradient"] = [0, E, np.abs(G).sum()]
    E, G = oracle.gradient_rows(X, F, F.shape[0] // 3, F.shape[0] // 2, nthreads=2)
    out["gradient_rows"] = [0, E, np.abs(G).sum()]
    V = X.shape[0]
    out["gradient_at"] = [0, np.abs(oracle.gradient_at(X, F, np.array([0, V // 2, V - 1], np.int32), nthreads=2)).sum()]
    out["pair_count"] = [oracle.pair_count(F)]
    E, G = oracle.conf_gradient(X, F, Y, FY, nthreads=2)
    out["conf_gradient"] = [0, E, np.abs(G).sum()]
    E, G = oracle.gradient_quad(X, F, 6, nthreads=2)
    out["gradient_quad"] = [0, E, np.abs(G).sum()]
    E, G = oracle.gradient_p3(X10, F10, 3, nthreads=2)
    out["gradient_p3"] = [0, E, np.abs(G).sum()]
    perm = oracle.kd_order(X, F, 32)
    h = 1469598103934665603
    for v in perm.tolist():
        h = ((h ^ v) * 1099511628211) & (2**64 - 1)
    out["kd_order"] = [0, h]
    E, G, st = oracle.farfield(X, F, 1.0, 32, perm, nthreads=2)
    out["farfield"] = [0, E, np.abs(G).sum(), st[0], st[1], st[2]]
    out["farfield_coverage"] = [0, *oracle.farfield_coverage(X, F, 1.0, 32, perm)]
    s = oracle.farfield_samples(X, F, 1.0, 7, 0.5, 1 << 20, 32, perm)
    n = len(s["block"])
    out["farfield_samples"] = [n, n, np.abs(s["feats"]).sum(), np.abs(s["targets"]).sum()]
    E, G, st = oracle.farfield_dual(X, F, 1.0, 32, perm, nthreads=2)
    out["farfield_dual"] = [0, E, np.abs(G).sum(), st[0], st[1]]
    perm3 = oracle.kd_order_p3(X10, F10, 3, 8)
    h = 1469598103934665603
    for v in perm3.tolist():
        h = ((h ^ v) * 1099511628211) & (2**64 - 1)
    out["kd_order_p3"] = [0, h]
    E, G, st = oracle.farfield_p3(X10, F10, 1.0, 3, leaf=8, perm=perm3, nthreads=2)
    out["farfield_p3"] = [0, E, np.abs(G).sum(), st[0], st[1], st[2]]
    out["farfield_coverage_p3"] = [0, *oracle.farfield_coverage_p3(X10, F10, 1.0, 3, leaf=8, perm=perm3)]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    try:
        oracle.build_sanitized(exe)
    except (subprocess.CalledProcessError, FileNotFoundError) as e:  # pragma: no cover
        pytest.skip(f"gcc cannot build with the sanitizers here: {e}")
    X, F = M.icosphere(3)
    X, _, _ = M.bump(X, 0, 0.3, 0.2)
    _, _, Y, FY = M.confinement_config(2, 2)
    X10, F10 = M.p3_sphere(1, 2, 4, 0.05, 0)
    _write(tmp_path / "mesh.bin", X, F)
    _write(tmp_path / "conf.bin", Y, FY)
    _write(tmp_path / "p3.bin", X10, F10)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    got = {}
    for line in r.stdout.splitlines():
        name, *vals = line.split()
        got[name] = [float(v) for v in vals]
    ref = _regular(X, F, Y, FY, X10, F10)
    assert set(got) == set(ref)
    assert got["farfield_samples"][0] > 0 and got["farfield"][3] > 0  # the cluster paths ran
    for name, vals in ref.items():
        assert len(got[name]) == len(vals), name
        for a, b in zip(got[name], vals):
            assert a == pytest.approx(float(b), rel=1e-12, abs=0.0), (name, got[name], vals)
