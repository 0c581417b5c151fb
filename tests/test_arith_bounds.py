"""The inner-loop arithmetic the kernels share with the host (short-quotient
integer butterflies, FP64 butterflies for primes below 2^50, carry-free
base-conversion sums: csrc/wide_arith.hpp), checked on the CPU against exact
128-bit arithmetic, including whole transforms with the kernels' reduction
points and every intermediate range (tests/native/arith_check.cpp, built
with hipcc for the host only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not available")
def test_kernel_arithmetic_bounds(tmp_path):
    exe = str(tmp_path / "arith_check")
    src = os.path.join(HERE, "native", "arith_check.cpp")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O2", "-ffp-contract=off", "-Wall",
                    "-Werror", src, "-o", exe], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("arith ok"), r.stdout + r.stderr
