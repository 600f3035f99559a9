"""CPU checks of the library's host arithmetic (no GPU): the near-field
regularizing polynomial (Section 3.1) matches the kernel, and the primal
cost's kernel, with their first two derivatives at the near-field radius,
for rho = 1 and real exponents.  The check program includes the library's
own header and is compiled here with the host compiler."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2201_07524_amd", "csrc")


def _build(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path / "host_math_check")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC,
                           "-o", exe, os.path.join(HERE, "host_math_check.cpp")])
    return exe


def test_nearfield_polynomial_matches_kernel_and_derivatives(tmp_path):
    out = subprocess.check_output([_build(tmp_path)], text=True)
    rows = [dict(kv.split("=") for kv in line.split()) for line in out.strip().splitlines()]
    assert len(rows) == 8
    for r in rows:
        # p = 8 matched derivatives: value and first two derivatives agree to
        # the finite-difference error (h = 1e-4 eI; for rho = 1, eI/e = 15
        # makes the kernel stiff and the second difference amplifies the
        # polynomial's 1e-12 rounding by (eI/h)^2), while a wrong term in the
        # construction gives mismatches of order one
        assert float(r["d0"]) <= 1e-10, r
        assert float(r["d1"]) <= 1e-6, r
        assert float(r["d2"]) <= 2e-3, r
        assert abs(float(r["p0"])) < 1e6, r
