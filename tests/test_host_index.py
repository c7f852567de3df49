"""The kernels' index arithmetic, checked exhaustively on the CPU.

tests/host_index_check.hip includes the library's device headers, builds for the
host only, and compares the shared neighbour helpers and the 4^4 SAP kernel's
per-thread setup (block of a workgroup, in-block neighbours, halo sites and their
boundary wraps) with plain coordinate arithmetic on every site of several
lattices.  No GPU is involved.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_index_arithmetic_exhaustive(tmp_path):
    exe = tmp_path / "host_index_check"
    src = os.path.join(ROOT, "tests", "host_index_check.hip")
    build = subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", src, "-o", str(exe)],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ALL OK")
