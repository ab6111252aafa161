"""The C ABI from C: tests/c_abi_check.c is compiled as C99 with gcc against
include/svd2.h, linked to libsvd2.so, and run.  It exercises the argument
checks, workspace queries and setters of every family of entry points, all of
which answer on the host (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2005_07403_amd", "libsvd2.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_c99_caller(tmp_path):
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("needs gcc and the HIP headers")
    assert os.path.exists(LIB), "build libsvd2.so first"
    exe = str(tmp_path / "c_abi_check")
    # the HIP headers select their AMD definitions by this macro (hipcc sets it itself)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror=implicit-function-declaration",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           "-o", exe, os.path.join(ROOT, "tests", "c_abi_check.c"), LIB,
           "-Wl,-rpath," + os.path.dirname(LIB)]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "all checks passed" in r.stdout
