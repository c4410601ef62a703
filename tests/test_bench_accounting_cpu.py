"""The benchmark's work accounting, on the CPU.

The roofline fractions that bench.py reports divide an algorithmic FLOP count
by a measured time.  These tests tie that count to the method: the routing
counts come from a closed-form trace of the galaxy covariance, checked here
against the oracle's covariances and route weights (Section 2, steps 3-4),
and the per-stamp totals on the throughput and differentiation workloads are
the figures the design notes quote.
"""

import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle.render as orr  # noqa: E402
import workloads as wl  # noqa: E402


def test_routing_counts_match_the_oracle_route_weights():
    rng = np.random.Generator(np.random.PCG64(2024))
    for W in (16, 32, 64, 128, 256):
        gal = wl.draw_galaxies(rng, 300, W, 0, r_e_range=(0.3, W / 3.0))
        for amp_var in (wl.generate.exp6_table(rng), wl.generate.dev8_table(rng)):
            var = np.asarray(amp_var[1], np.float64)
            kf, kr = bench.routing_counts(gal, var, W)
            for i in range(len(gal.x)):
                a, _, d = orr.covariances(float(gal.r_e[i]), float(gal.e1[i]), float(gal.e2[i]), var)
                w = orr.routing_weights(a, d, W)
                assert kf[i] == int((w > 0).sum()), (W, i)
                assert kr[i] == int((w < 1).sum()), (W, i)


def test_per_stamp_counts_follow_the_step_counts():
    # W = 16, one Fourier component, none in real space: 171 evaluation
    # points (the 144 bins of the half spectrum with the Nyquist column, the
    # Nyquist row's 9 twins at omega = -1/2, the Nyquist column's 16 rows at
    # the other sign of nu, 2 corner twins), 2.5 W^2 log2 W^2 for the FFT
    W, H = 16, 16 * 9
    n_eval = H + 9 + 16 + 2
    fft = 2.5 * W * W * math.log2(W * W)
    assert bench.algorithmic_flops_per_stamp(W, np.array([1]), np.array([0]))[0] == n_eval * 8 + 14 * H + fft
    assert bench.adjoint_flops_per_stamp(W, np.array([1]), np.array([0]))[0] == n_eval * 27 + 14 * H + fft
    # each real-space component adds its per-pixel work over the whole stamp
    d_fwd = bench.algorithmic_flops_per_stamp(W, np.array([1]), np.array([1]))[0] - \
        bench.algorithmic_flops_per_stamp(W, np.array([1]), np.array([0]))[0]
    assert d_fwd == 7 * W * W


def test_workload_means_are_the_quoted_figures():
    cfg = wl.config_metric()
    per = bench.workload_flops(cfg["gal"], cfg["mix"], 64) / len(cfg["gal"].x)
    assert abs(per - 246_880) < 1.0
    cfg = wl.config5()
    per = bench.workload_flops(cfg["gal"], cfg["mix"], 64, adjoint=True) / len(cfg["gal"].x)
    assert abs(per - 358_008) < 1.0


def test_traffic_record_is_used_only_for_the_sources_it_was_taken_from(tmp_path, monkeypatch):
    import hashlib

    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    rec = tmp_path / "traffic.txt"
    rec.write_text(f"kernel: k\nsource_sha256_16: {h}\nsources: k.hip\n"
                   "fetch_bytes_per_launch: 100\nwrite_bytes_per_launch: 2000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic() == 2100.0
    src.write_text("kernel source, changed\n")
    assert bench.measured_traffic() is None
    src.unlink()
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
