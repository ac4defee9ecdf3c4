"""The symmetric pair kernel's schedule arithmetic, checked on the host under AddressSanitizer and
UndefinedBehaviorSanitizer (tests/native/sched_check.cpp: range tiling, inverse lookups, costs and
column partial counts over many sizes, widths and work-group counts).  The device code of pair.hip
is compiled as usual but never launched, so no GPU is needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_schedule_arithmetic_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):  # pragma: no cover
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "sched_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-I" + os.path.join(ROOT, "paper_2509_22110_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "native", "sched_check.cpp"),
           os.path.join(ROOT, "paper_2509_22110_amd", "csrc", "pair.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    assert " 0 failures" in r.stdout
