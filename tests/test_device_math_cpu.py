"""The kernels' sin/cos of pi r (gfc::sincospi_poly, a Taylor polynomial on
|f| <= 1/4 after reduction by half turns) compiled for the host and checked
against double-precision sin/cos: absolute error below 1.5e-7 over a dense
sweep of |r| <= 512 (the phases the kernels form) and a random sample,
exact values at integer and half-integer r, and odd/even symmetry bit for
bit (the kernels take the omega = -1/2 phase as the conjugate of the
omega = +1/2 one)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_sincospi_poly_accuracy(tmp_path):
    exe = tmp_path / "sincospi_check"
    cmd = ["hipcc", "-O2", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2012_15797_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "sincospi_check.hip"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=300).stdout.split()
    err_s, err_c, bad_exact, bad_sym = float(out[0]), float(out[1]), int(out[2]), int(out[3])
    assert err_s < 1.5e-7 and err_c < 1.5e-7, (err_s, err_c)
    assert bad_exact == 0
    assert bad_sym == 0
