"""Device arithmetic compiled for the host and checked against double precision.

- gfc::sincospi_poly (sin/cos of pi r, a Taylor polynomial on |f| <= 1/4
  after reduction by half turns): absolute error below 1.5e-7 over a dense
  sweep of |r| <= 512 (the phases the kernels form) and a random sample,
  exact values at integer and half-integer r, and odd/even symmetry bit for
  bit (the kernels take the omega = -1/2 phase as the conjugate of the
  omega = +1/2 one).
- gfc::fft<N, SIGN>, the in-register FFTs of every kernel."""

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


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_register_fft_accuracy(tmp_path):
    """The kernels' in-register FFTs (gfc::fft<N, SIGN>: decimation-in-time
    stages whose twiddles are written as a real scale times (1 + i tan) or
    (cot + i) and folded into FMA butterflies), compiled for the host and
    compared with a double-precision direct DFT of the same inputs at every
    power-of-two length 1..256 and both signs: error relative to the largest
    output below 4e-7 (a few float32 roundings per stage), and exact results
    for a unit impulse and a constant."""
    exe = tmp_path / "fft_check"
    cmd = ["hipcc", "-O2", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2012_15797_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "fft_check.hip"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    lines = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=300).stdout.splitlines()
    seen = set()
    for line in lines:
        n, sign, err, bad = line.split()
        seen.add((int(n), int(sign)))
        assert float(err) < 4e-7, line
        assert int(bad) == 0, line
    assert seen == {(1 << e, s) for e in range(9) for s in (1, -1)}
