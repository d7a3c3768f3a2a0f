"""The float64 near field's sine/cosine (csrc/phase64.h), compiled for the
host and checked against the C library's long-double sine and cosine on
[-200, 200] (2e6 points) and at quadrant boundaries: absolute error < 5e-16."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_sincos_reduced_matches_libm(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "phase64_check"
    res = subprocess.run([hipcc, "-O2", "-std=c++17", os.path.join(HERE, "cpp", "phase64_check.cpp"),
                          "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout
