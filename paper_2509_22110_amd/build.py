"""Build libtpe.so (HIP, gfx950 only) in-tree.

Every ``csrc/*.hip`` file is compiled with hipcc for gfx950 and linked into
``paper_2509_22110_amd/libtpe.so``.  Packed-FP32 code generation is switched off for all device
code (``-Xclang -target-feature -Xclang -packed-fp32-ops``): the kernels use scalar FP32 VALU
instructions only.

Usage:  python -m paper_2509_22110_amd.build     (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtpe.so")
# stand-alone measurement tool (not part of libtpe): FP32 VALU issue rates of the pair kernels' mixes
PROBE_SRC = os.path.join(PKG, "measure", "valu_issue.hip")
PROBE_BIN = os.path.join(PKG, "measure", "valu_issue")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in VGPRs (gfx950 allows either): the MLP's activations are read back by
    # VALU code after every layer, which from AGPRs costs one v_accvgpr_read per value
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *DEVICE_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def _build_probe() -> str:
    """Compile the VALU issue-rate tool (measure/valu_issue.hip) into an executable beside it."""
    cmd = [HIPCC, *[f for f in DEVICE_FLAGS if f != "-fPIC"], PROBE_SRC, "-o", PROBE_BIN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip()]
        raise RuntimeError("hipcc failed for " + PROBE_SRC + ":\n" + "\n".join(msgs))
    return PROBE_BIN


def build(jobs: int = 8) -> str:
    """Compile all HIP sources and link libtpe.so, and the measurement tool; always rebuilds.
    Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs) + 1))) as ex:
        probe = ex.submit(_build_probe)
        objs = list(ex.map(_compile, srcs))
        probe.result()
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
