#!/usr/bin/env python3
"""Throughput benchmark of the hybrid Fourier-real galaxy-PSF renderer.

Workload: 100,000 galaxies with a deVaucouleurs-like 8-component mixture
(synthetic table), 64x64 stamps, a 64x64 Moffat (beta=3, FWHM 4.5 px) + 1%
Gaussian-halo PSF, hybrid Fourier/real routing, parameters drawn with the
batched-render distributions (workloads.config_metric).

One step = one batched forward render of the whole batch (steps 3-8 of the
method, one fused kernel launch) with inputs resident in device memory.  The
PSF-FT cache is filled before timing (a cold, once-per-PSF step) and timed
separately.  Printed: ONE JSON line (see the keys below).

Order of a run:
  1. CPU leg (before the GPU is touched): the FP64 oracle, one single-threaded
     process per core of this process's CPU share, timed on a seeded sample
     of the workload (cpu_baseline); the same processes then compute, untimed,
     the reference samples that gate every other reported number.
  2. Rate probes of the device (FMA, v_exp_f32, HBM write and copy): the
     measured roofline denominators.
  3. Settle steps (at least 45 and 50 ms of device time): a GPU that was
     idle runs a few launches of this full load fast, is then throttled by
     its power management (about 0.75 ms per launch instead of 0.52) and
     reaches steady clocks after about 25 ms.  These untimed steps carry it
     through that transient, then W warm-up steps, then K timed steps (HIP
     events on the launch stream).
  4. Parity of the timed output, the plain per-request launches, serving,
     and the other workloads, each with a parity record from its own launch.
     Each other workload is timed after untimed launches of its own by the
     same rule.

    python bench.py [--gpus 1] [--steps 100] [--warmup 30] [--settle 45] [--settle-ms 50]
"""

from __future__ import annotations

import argparse
import io
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

METRIC = "stamps/sec (64², K=8 MoG) batched vs plain at ≤1e-5 peak err; p99 latency"

# MI355X peaks used for the roofline (published / derived from unit counts).
CU, SIMD_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
FP32_FMA_NONPACKED_TFLOPS = CU * SIMD_PER_CU * LANES_PER_SIMD * 2 * CLOCK_HZ / 1e12   # 78.6
FP32_PUBLISHED_TFLOPS = 157.3   # counts packed FP32 FMAs, which this build does not use
HBM_GBPS = 8000.0
TOL_PEAK = 1e-5                 # forward parity bar: max |gpu - oracle| <= TOL_PEAK x peak
CPU_SHARE = 16                  # host CPUs that go with one GPU

KQ = -2.0 * math.pi**2 * math.log2(math.e)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- work accounting
def routing_counts(gal, var, W):
    """K_F (components with Fourier weight > 0) and K_R (weight < 1) per galaxy,
    from the closed-form pixel covariance trace: tr C_i = v_i r_e^2 (2 + 2 e^2)/(1 + e)^2.
    var: the components' variances [K], or per galaxy [n][K]."""
    r = gal.r_e.astype(np.float64)
    e = np.hypot(gal.e1.astype(np.float64), gal.e2.astype(np.float64))
    tr = r * r * (2.0 + 2.0 * e * e) / (1.0 + e) ** 2
    var = np.asarray(var, np.float64)
    n = (W / 2.0) / np.sqrt((var[None, :] if var.ndim == 1 else var) * tr[:, None])
    kf = (n > 3.0).sum(axis=1)
    kr = (n < 4.0).sum(axis=1)
    return kf, kr


def algorithmic_flops_per_stamp(W, kf, kr):
    """FLOPs the method needs per stamp (FMA = 2, other ops and exp = 1):
    the mixture transform on the half spectrum plus the Nyquist duplicates
    (quadratic form 4, per Fourier component: scale 1 + exp 1 + accumulate 2),
    phase x PSF x flux (14 per bin), the complex-to-real 2-D inverse FFT
    (2.5 W^2 log2 W^2), and real-space components (7 per pixel each)."""
    H = W * (W // 2 + 1)
    n_eval = H + (W // 2 + 1) + W + 2
    return n_eval * (4.0 + 4.0 * kf) + 14.0 * H + 2.5 * W * W * math.log2(W * W) + 7.0 * W * W * kr


def adjoint_flops_per_stamp(W, kf, kr):
    """FLOPs the adjoint needs per stamp (FMA = 2, exp = 1): the real-to-complex
    2-D transform of the upstream gradient (2.5 W^2 log2 W^2); per evaluation
    point the PSF x phase x conj(G) product (14) and the parameter sums from
    the bin's S and S1 (19: flux, two positions, three shape entries); per
    Fourier component and point an exponential, its scale and three
    accumulations (S, S1, the component's own sum: 8); per real-space
    component and pixel the value and the six parameter accumulations (11)."""
    H = W * (W // 2 + 1)
    n_eval = H + (W // 2 + 1) + W + 2
    return n_eval * (19.0 + 8.0 * kf) + 14.0 * H + 2.5 * W * W * math.log2(W * W) + 11.0 * W * W * kr


def workload_flops(gal, mix, W, adjoint=False):
    """Algorithmic FLOPs of one launch over `gal` (stamp size W), from each
    galaxy's routing counts under its own mixture table."""
    mid = np.asarray(gal.mix_id) if getattr(gal, "mix_id", None) is not None else np.zeros(len(gal.x), np.int32)
    mid = np.broadcast_to(mid, (len(gal.x),))
    f = adjoint_flops_per_stamp if adjoint else algorithmic_flops_per_stamp
    total = 0.0
    for t in np.unique(mid):
        sel = np.nonzero(mid == t)[0]
        k = int(mix.K[t])
        kf, kr = routing_counts(gal.subset(sel), np.asarray(mix.var[t, :k], np.float64), W)
        total += float(f(W, kf, kr).sum())
    return total


def pergal_flops(gal, var, W):
    """Algorithmic FLOPs of one forward launch whose galaxy i has its own
    component variances var[i] (the interpolated Sersic and the bulge + disk
    mixtures)."""
    kf, kr = routing_counts(gal, var, W)
    return float(algorithmic_flops_per_stamp(W, kf, kr).sum())


def eigen_psf_flops(W, J):
    """FLOPs per stamp of forming a varying PSF's spectrum from J component
    spectra (a real weight times a complex value, accumulated: 4 per
    component and bin of the half spectrum and Nyquist column)."""
    return 4.0 * J * (W * (W // 2 + 1) + W)


def lanczos_flops(W):
    """FLOPs per stamp of the separable six-tap Lanczos-3 shift (an FMA per
    tap along x, then along y)."""
    return 24.0 * W * W


def settle_device(fn, min_launches, min_ms, batch=8, max_launches=200_000):
    """Runs fn untimed until at least min_launches launches and min_ms of
    device time (HIP events over batches of launches) have passed; returns
    the number of launches.  A device that was idle goes through a
    power-management transient (a fast start, a throttled stretch, then
    steady clocks) that takes tens of milliseconds of full load, whatever
    the length of one launch."""
    import torch

    n, t = 0, 0.0
    while (n < min_launches or t < min_ms) and n < max_launches:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(batch):
            fn()
        b.record()
        b.synchronize()
        t += a.elapsed_time(b)
        n += batch
    return n


def flops_roofline(flops, ms):
    """Achieved TFLOP/s of a launch and its fraction of the FP32 FMA peak
    without packed instructions."""
    tf = flops / (ms * 1e-3) / 1e12
    return dict(bound="alu", achieved_tflops=round(tf, 3), peak_tflops=round(FP32_FMA_NONPACKED_TFLOPS, 2),
                frac=round(tf / FP32_FMA_NONPACKED_TFLOPS, 4), flops_per_launch=round(flops, 1))


def algorithmic_issue_slots(W, kf, kr):
    """(VALU issue slots, exponentials) per stamp of the same algorithm when
    every FMA-able pair is one instruction: quadratic form 2 per evaluation
    point, per Fourier component a multiply, an exponential and an FMA; 10
    per bin for phase x PSF x flux; (5/3) W^2 log2 W^2 for the inverse FFT
    with FMA butterflies (2.5 W^2 log2 W^2 FLOP at 1.5 FLOP per slot);
    per real-space component and pixel two FMAs, an exponential and an FMA."""
    H = W * (W // 2 + 1)
    n_eval = H + (W // 2 + 1) + W + 2
    slots = n_eval * (2.0 + 3.0 * kf) + 10.0 * H + (5.0 / 3.0) * W * W * math.log2(W * W) + 4.0 * W * W * kr
    exps = n_eval * kf + W * W * kr
    return slots, exps


# ---------------------------------------------------------------- HBM traffic record
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_render_small_kernel_64.txt")


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel sources have changed since
    the counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in rec.get("sources", "").split(","):
        path = os.path.join(ROOT, f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])


# ---------------------------------------------------------------- CPU leg: the oracle
# Reference samples gating the other reported numbers: (job, workload size, sample size).
REF_JOBS = {
    "mixed": 120, "large": 24, "lanczos": 48, "sersic": 48, "composite": 48, "eigen": 36, "backward": 24,
}
BWD_NOISE_SEED = wl.SEED_BASE + 55    # upstream gradient of the adjoint line: unit-normal noise


def serving_traces(seconds):
    """(label, rate, seconds, restricted) of the replayed traces: the full
    serving configuration (64 PSFs, stamps 16..256) at its nominal rate and
    at ten times that, and the 64x64 one-PSF variant at the nominal and the
    tenfold rate."""
    return (("", 2000.0, seconds, False), ("saturated_", 20000.0, min(seconds, 2.0), False),
            ("restricted64_", 2000.0, min(seconds, 3.0), True),
            ("saturated64_", 20000.0, min(seconds, 1.0), True))


def serving_sample(requests):
    """Requests whose stamps gate a replay: per stamp size, two seeded
    requests of at most 256 galaxies, and their first three galaxies."""
    rng = np.random.Generator(np.random.PCG64(7100))
    out = []
    for W in sorted({r["W"] for r in requests}):
        cand = [i for i, r in enumerate(requests) if r["W"] == W and len(r["gal"]) <= 256]
        for i in sorted(rng.choice(cand, min(2, len(cand)), replace=False).tolist()):
            out.append((i, list(range(min(3, len(requests[i]["gal"]))))))
    return out


def ref_indices(job, n_total, k):
    """Seeded sample of a workload; for the mixed and large workloads it is
    stratified by stamp size (equal numbers per size)."""
    rng = np.random.Generator(np.random.PCG64(7000 + sorted(REF_JOBS).index(job)))
    if job in ("mixed", "large"):
        cfg = wl.config2() if job == "mixed" else wl.config3()
        Ws = sorted(set(int(w) for w in cfg["gal"].W))
        per = k // len(Ws)
        idx = []
        for W in Ws:
            idx += rng.choice(np.nonzero(cfg["gal"].W == W)[0], per, replace=False).tolist()
        return np.array(sorted(idx))
    return np.sort(rng.choice(n_total, k, replace=False))


def _oracle_job(job, idx, n_metric, serve_spec=None):
    """The oracle's stamps (or gradients) for one reference job; a serving
    job returns the stamps of its trace's sample in order (idx numbers them)."""
    import oracle as o
    from oracle import eigen as oe
    from oracle import lanczos as ol
    from oracle import sersic as osr

    if job == "metric":
        cfg = wl.config_metric(n_metric)
        return o.render_batch(cfg["psf"].astype(np.float64), cfg["mix"].as_f32(), cfg["gal"], idx=idx)
    if job in ("mixed", "large"):
        cfg = wl.config2() if job == "mixed" else wl.config3()
        return o.render_batch(cfg["psf"].astype(np.float64), cfg["mix"].as_f32(), cfg["gal"],
                              psf_gauss=cfg.get("psf_gauss"), idx=idx)
    if job == "lanczos":
        cfg = wl.config_metric()
        P = cfg["psf"].astype(np.float64)
        ph, g = o.psf_spectrum(P, 64), o.psf_gauss_moments(P)
        amp, var = cfg["mix"].as_f32().table(0)
        out = []
        for i in idx:
            p = cfg["gal"].params(int(i))
            out.append(ol.render_stamp_lanczos(ph, g, amp, var, p["x"], p["y"], p["flux"], p["r_e"], p["e1"],
                                               p["e2"], 64, 8))
        return out
    if job == "sersic":
        cfg = wl.config_sersic()
        fam = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in cfg["family"].items()}
        return osr.render_batch_sersic(cfg["psf"].astype(np.float64), fam, cfg["gal"], cfg["sersic_n"], idx=idx)
    if job == "composite":
        cfg = wl.config_composite()
        P = cfg["psf"].astype(np.float64)
        ph, g = o.psf_spectrum(P, 64), o.psf_gauss_moments(P)
        m = cfg["mix"].as_f32()
        (ad, vd), (ab, vb) = m.table(0), m.table(1)
        out = []
        for i in idx:
            p = cfg["gal"].params(int(i))
            a, v = osr.composite_mixture(ad, vd, ab, vb, float(cfg["bulge_frac"][i]), float(cfg["bulge_rho"][i]))
            out.append(o.render_stamp(ph, g, a, v, p["x"], p["y"], p["flux"], p["r_e"], p["e1"], p["e2"], 64))
        return out
    if job == "eigen":
        cfg = wl.config_eigen()
        eig = dict(cfg["eig"], comps=np.asarray(cfg["eig"]["comps"], np.float32).astype(np.float64))
        return oe.render_batch_eigen(eig, cfg["mix"].as_f32(), cfg["gal"], cfg["psf_x"], cfg["psf_y"], idx=idx)
    if job == "backward":
        cfg = wl.config5()
        P = cfg["psf"].astype(np.float64)
        ph, g = o.psf_spectrum(P, 64), o.psf_gauss_moments(P)
        amp, var = cfg["mix"].as_f32().table(0)
        noise = wl.generate.noise_field(BWD_NOISE_SEED, len(cfg["gal"]), 64)
        out = []
        for i in idx:
            p = cfg["gal"].params(int(i))
            _, J = o.render_stamp_jacobian(ph, g, amp, var, p["x"], p["y"], p["flux"], p["r_e"], p["e1"],
                                           p["e2"], 64)
            lg = o.loss_gradient(noise[i].astype(np.float64), J)
            out.append(np.array([lg[k] for k in ("x", "y", "flux", "log_re", "e1", "e2")]))
        return out
    if job.startswith("serving"):
        label, rate, secs, restricted = serve_spec[job]
        tr = wl.config4_trace(duration_s=secs, rate_hz=rate, restricted=restricted)
        m = tr["mix"].as_f32()
        out = []
        for ri, gis in serving_sample(tr["requests"]):
            r = tr["requests"][ri]
            P = np.asarray(tr["psfs"][r["psf"]], np.float32).astype(np.float64)
            ph, g = o.psf_spectrum(P, r["W"]), o.psf_gauss_moments(P)
            for gi in gis:
                p = r["gal"].params(gi)
                amp, var = m.table(p["mix_id"])
                out.append(o.render_stamp(ph, g, amp, var, p["x"], p["y"], p["flux"], p["r_e"], p["e1"], p["e2"],
                                          r["W"]))
        return out
    raise ValueError(job)


def oracle_worker_main():
    """`bench.py --oracle-worker`: reads a job list (JSON) on stdin, runs the
    oracle single-threaded and writes an .npz to stdout."""
    spec = json.loads(sys.stdin.read())
    import threadpoolctl

    res = {}
    with threadpoolctl.threadpool_limits(1):
        for job, idx, timed in spec["jobs"]:
            t0 = time.perf_counter()
            out = _oracle_job(job, [int(i) for i in idx], spec["n_metric"], spec.get("serve"))
            dt = time.perf_counter() - t0
            keys = range(len(out)) if job.startswith("serving") else idx   # a serving job numbers its stamps
            for i, a in zip(keys, out):
                res[f"{job}/{i}"] = np.asarray(a, np.float64)
            if timed:
                res[f"__cpu_s__/{job}/{idx[0]}"] = np.array(dt)
    buf = io.BytesIO()
    np.savez(buf, **res)
    sys.stdout.buffer.write(buf.getvalue())
    sys.stdout.buffer.flush()


def _run_workers(job_lists, n_metric, serve=None):
    """One child process per job list; returns (merged results, wall s).
    Every child is waited for, so none outlives the call."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    t0 = time.perf_counter()
    procs = []
    for jobs in job_lists:
        p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker"], stdin=subprocess.PIPE,
                             stdout=subprocess.PIPE, env=env)
        procs.append(p)
    outs = []
    try:
        for p, jobs in zip(procs, job_lists):
            p.stdin.write(json.dumps(dict(jobs=jobs, n_metric=n_metric, serve=serve)).encode())
            p.stdin.close()
        for p in procs:
            data = p.stdout.read()
            rc = p.wait()
            if rc != 0:
                raise RuntimeError(f"oracle worker exited with {rc}")
            outs.append(data)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
    wall = time.perf_counter() - t0
    merged = {}
    for data in outs:
        with np.load(io.BytesIO(data)) as z:
            for k in z.files:
                merged[k] = z[k]
    return merged, wall


def cpu_leg(n_metric, sample, workers, other, serve_seconds=0.0):
    """The oracle, unchanged, timed on a seeded sample of the metric workload
    in `workers` single-threaded processes (cpu_baseline); then the untimed
    reference samples of the other numbers.  Runs before the GPU is touched."""
    rng = np.random.Generator(np.random.PCG64(2024))
    idx = np.sort(rng.choice(n_metric, size=sample, replace=False))
    lists = [[["metric", c.tolist(), True]] for c in np.array_split(idx, workers)]
    res, wall = _run_workers(lists, n_metric)
    times = [float(v) for k, v in res.items() if k.startswith("__cpu_s__")]
    cpu_s, span = sum(times), max(times)
    metric_refs = {int(k.split("/")[1]): v for k, v in res.items() if k.startswith("metric/")}
    host_cpus = os.cpu_count() or 1
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else host_cpus
    cpu = dict(value=round(sample / span, 1), unit="stamps/s", cores=workers, kind="oracle",
               host_cpu_count=host_cpus, cpus_available=share,
               sample=f"{sample} seeded stamps of the 100k workload, FP64 oracle, {workers} single-threaded "
                      f"processes (host os.cpu_count() {host_cpus}, {share} CPUs in this process's affinity, "
                      f"of which one GPU's share is {CPU_SHARE}); {cpu_s:.1f} CPU-s, the slowest process "
                      f"{span:.2f} s in the oracle (value = sample / that), {wall:.2f} s wall with start-up")
    refs = {}
    serve = {f"serving_{label or 'full_'}": [label, rate, secs, restricted]
             for label, rate, secs, restricted in serving_traces(serve_seconds)} if serve_seconds > 0 else {}
    if other or serve:
        jobs = [[job, [0], False] for job in serve]   # one job per trace (it draws the whole trace)
        for job, k in (REF_JOBS.items() if other else ()):
            n_total = {"lanczos": 100_000, "sersic": 100_000, "composite": 100_000, "eigen": 100_000,
                       "backward": 10_000}.get(job, 0)
            ii = ref_indices(job, n_total, k)
            refs[job] = ii
            for c in np.array_split(ii, max(1, min(workers, len(ii) // 4))):
                if len(c):
                    jobs.append([job, c.tolist(), False])
        lists = [jobs[i::workers] for i in range(workers) if jobs[i::workers]]
        res2, wall2 = _run_workers(lists, n_metric, serve)
        refs = {job: (ii, [res2[f"{job}/{i}"] for i in ii]) for job, ii in refs.items()}
        for job in serve:   # a serving job's stamps come back numbered 0, 1, ...
            k = sum(1 for key in res2 if key.startswith(job + "/"))
            refs[job] = [res2[f"{job}/{i}"] for i in range(k)]
        log(f"cpu leg: reference samples for {len(refs)} workloads in {wall2:.1f} s")
    return cpu, metric_refs, refs


def stamp_parity(gpu_rows, ref_rows):
    errs = [float(np.abs(g - r).max() / np.abs(r).max()) for g, r in zip(gpu_rows, ref_rows)]
    return dict(n_checked=len(errs), max_err_over_peak=max(errs), tol=TOL_PEAK,
                passed=bool(max(errs) <= TOL_PEAK))


# ---------------------------------------------------------------- device rate probes
def rate_probes(dev):
    """Measured denominators: FP32 FMA issue rate, v_exp_f32 alone and
    interleaved with FMAs, streamed HBM write and copy."""
    import ctypes

    import torch

    path = os.path.join(ROOT, "paper_2012_15797_amd", "libgfc_microbench.so")
    mb = ctypes.CDLL(path)
    D = ctypes.POINTER(ctypes.c_double)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    sink = torch.zeros(4, device=dev)
    sp = ctypes.c_void_p(sink.data_ptr())
    out = {}

    def chk(rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} probe failed: {rc}")

    v = ctypes.c_double()
    mb.gfc_mb_fma.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, D]
    chk(mb.gfc_mb_fma(5, sp, stream, ctypes.byref(v)), "fma")
    fma = v.value
    out["fp32_fma_tflops"] = round(2 * fma / 1e12, 2)
    mb.gfc_mb_exp.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, D]
    chk(mb.gfc_mb_exp(5, sp, stream, ctypes.byref(v)), "exp")
    out["exp_only_g_per_s"] = round(v.value / 1e9, 1)
    out["exp_only_fma_slots"] = round(fma / v.value, 3)
    mb.gfc_mb_exp_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, D, D]
    mixed = {}
    for F in (1, 2, 3, 4):
        e, f = ctypes.c_double(), ctypes.c_double()
        chk(mb.gfc_mb_exp_fma(F, 5, sp, stream, ctypes.byref(e), ctypes.byref(f)), "exp+fma")
        # issue slots one exponential costs beside F FMAs, in units of one FMA's slot
        mixed[F] = round(fma / e.value - F, 3)
    out["exp_fma_slots_with_F_fmas"] = mixed
    nbytes = 2 << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    mb.gfc_mb_hbm_write.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p, D]
    chk(mb.gfc_mb_hbm_write(ctypes.c_void_p(b.data_ptr()), nbytes, 5, stream, ctypes.byref(v)), "write")
    out["hbm_write_gbps"] = round(v.value / 1e9, 1)
    mb.gfc_mb_hbm_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p, D]
    chk(mb.gfc_mb_hbm_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), nbytes, 5, stream,
                           ctypes.byref(v)), "copy")
    out["hbm_copy_gbps"] = round(v.value / 1e9, 1)
    del a, b
    torch.cuda.synchronize()
    return out


# ---------------------------------------------------------------- main
def main():
    if "--oracle-worker" in sys.argv:
        oracle_worker_main()
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--settle", type=int, default=45,
                    help="least number of untimed steps before the warm-up that carry the device through its "
                         "power-management transient (a fast start, a throttled stretch, then steady clocks after "
                         "about 25 ms of full load); the count run is reported as settle_steps")
    ap.add_argument("--settle-ms", type=float, default=50.0,
                    help="least device time of those settle steps (and of each other case's untimed launches)")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--cpu-sample", type=int, default=20000)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the mixed-size, 64-PSF Poisson request trace replayed against the "
                         "server, batched and plain (0: skip serving)")
    ap.add_argument("--no-other", action="store_true", help="skip the other-workload throughput table")
    ap.add_argument("--no-probes", action="store_true", help="skip the device rate probes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--profile-set", action="store_true",
                    help="only launch every kernel instantiation a few times (for rocprofv3) and print "
                         "their launch times")
    ap.add_argument("--profile-reps", type=int, default=3)
    ap.add_argument("--profile-settle", type=int, default=0,
                    help="untimed launches of each --profile-set case before its timed ones")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this renderer runs on one GPU; --gpus must be 1 "
              "(stamps are independent, so more GPUs would each take a shard of the batch)",
              file=sys.stderr)
        sys.exit(2)

    if args.profile_set:
        import torch

        import paper_2012_15797_amd as gfc

        dev = torch.device("cuda", 0)
        res = profile_set(gfc, gfc.Context.default(0), dev, args.profile_reps, args.profile_settle)
        if args.copy_calibration:
            a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
            b = torch.empty_like(a)
            a.fill_(1.0)
            torch.cuda.synchronize()
            b.copy_(a)
            torch.cuda.synchronize()
            log("copy calibration: 1 GiB read + 1 GiB written")
        print(json.dumps(dict(profile_set=res)), flush=True)
        return

    cfg = wl.config_metric(args.n)
    gal = cfg["gal"]
    W = 64
    mixf = cfg["mix"].as_f32()
    amp, var = mixf.table(0)
    kf, kr = routing_counts(gal, var, W)
    flops_stamp = algorithmic_flops_per_stamp(W, kf, kr)

    cpu, oracle_stamps, refs = None, {}, {}
    if not args.no_cpu_baseline:
        share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        workers = args.cpu_workers or max(1, min(CPU_SHARE, share))
        log(f"cpu leg: oracle on {args.cpu_sample} stamps with {workers} processes")
        cpu, oracle_stamps, refs = cpu_leg(args.n, args.cpu_sample, workers, not args.no_other, args.serve_seconds)
        log(f"cpu baseline: {cpu['value']:.1f} stamps/s")

    import torch

    import paper_2012_15797_amd as gfc

    dev = torch.device("cuda", 0)
    probes = None if args.no_probes else rate_probes(dev)
    if probes:
        log(f"rate probes: {probes}")
    ctx = gfc.Context.default(0)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, mixf)
    d = lambda a: torch.as_tensor(a).to(dev)
    x, y, fl, re, e1, e2 = map(d, (gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2))
    out = torch.empty((args.n, W, W), dtype=torch.float32, device=dev)

    t0 = time.perf_counter()
    psf.prepare(W)
    torch.cuda.synchronize()
    psf_cache_ms = (time.perf_counter() - t0) * 1e3

    def step():
        gfc.gfc_render_stamps(ctx, psf, mix, x, y, fl, re, e1, e2, W, out=out)

    # Settle: a full-load launch sequence on a freshly started GPU runs fast for
    # a few launches, is then throttled (about 0.75 ms per 64x64 launch instead
    # of 0.52) and recovers over about 40 launches.  These untimed steps carry
    # the device through that transient, so the timed steps measure the steady
    # state at any --warmup.
    settle_steps = settle_device(step, args.settle, args.settle_ms)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"settle ({settle_steps} steps) and warmup ({args.warmup} steps) done")

    stream = torch.cuda.current_stream(dev)     # the stream the library launches on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t_start
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    ms_per_step = wall_s * 1e3 / args.steps
    value = args.n / (ms_per_step / 1e3)
    avg_kern_ms = float(kern_ms.mean())
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, kernel mean {avg_kern_ms:.3f} ms, "
        f"median {np.median(kern_ms):.3f}, min {kern_ms.min():.3f}")
    log("kernel ms per timed step: " + " ".join(f"{v:.3f}" for v in kern_ms))

    flops_launch = float(flops_stamp.sum())
    achieved_tflops = flops_launch / (avg_kern_ms * 1e-3) / 1e12
    roofline = dict(bound="alu", achieved=round(achieved_tflops, 3), peak=round(FP32_FMA_NONPACKED_TFLOPS, 2),
                    unit="TFLOP/s", frac=round(achieved_tflops / FP32_FMA_NONPACKED_TFLOPS, 4),
                    traffic=measured_traffic(),
                    kernel="render_small_kernel<64, false, false, false>",
                    flops_per_stamp=round(float(flops_stamp.mean()), 1),
                    peak_note="FP32 vector FMA peak without packed instructions: 256 CU x 4 SIMD x 16 lanes x "
                              "2 FLOP x 2.4 GHz",
                    published_peak=FP32_PUBLISHED_TFLOPS,
                    frac_published=round(achieved_tflops / FP32_PUBLISHED_TFLOPS, 4),
                    achieved_median_time=round(flops_launch / (float(np.median(kern_ms)) * 1e-3) / 1e12, 3),
                    algorithmic_bytes=args.n * (4 * W * W + 28),
                    hbm_gbps=round(args.n * (4 * W * W + 28) / (avg_kern_ms * 1e-3) / 1e9, 1),
                    hbm_frac=round(args.n * (4 * W * W + 28) / (avg_kern_ms * 1e-3) / 1e9 / HBM_GBPS, 4))
    if probes:
        meas = probes["fp32_fma_tflops"]
        roofline.update(measured_peak=meas, frac_measured=round(achieved_tflops / meas, 4),
                        hbm_measured_write_gbps=probes["hbm_write_gbps"])
        # issue-slot model with the measured cost of an exponential beside two FMAs (the mixture loop's mix)
        slots, exps = algorithmic_issue_slots(W, kf, kr)
        c_exp = probes["exp_fma_slots_with_F_fmas"][2]
        t_model = float((slots + (c_exp - 1.0) * exps).sum()) / (meas * 1e12 / 2.0)
        roofline["issue_model"] = dict(
            slots_per_stamp=round(float(slots.mean()), 1), exps_per_stamp=round(float(exps.mean()), 1),
            exp_cost_slots=c_exp, time_ms=round(t_model * 1e3, 4),
            frac=round(t_model / (avg_kern_ms * 1e-3), 4),
            note="time the algorithm's minimal VALU issue needs at the measured FMA rate, an exponential "
                 "costing the measured slots beside FMAs; frac = that time / kernel time")

    parity = None
    if oracle_stamps:
        idx = sorted(oracle_stamps)
        sel = out[torch.as_tensor(idx, device=dev)].cpu().numpy().astype(np.float64)
        parity = stamp_parity(sel, [oracle_stamps[i] for i in idx])
        log(f"parity on {len(idx)} stamps: max err/peak {parity['max_err_over_peak']:.2e}")

    plain = None
    if not args.no_plain:
        plain = plain_per_request(gfc, ctx, psf, mix, gal, W, dev, oracle_stamps)
        log(f"plain per-request launches: {plain['value']:.3e} stamps/s over {plain['requests']} requests")
    del out
    psf.close()
    mix.close()

    serving = None
    if args.serve_seconds > 0:
        serving = serving_benchmark(gfc, ctx, args.serve_seconds, refs)

    other = None
    if not args.no_other:
        other = size_throughput(gfc, ctx, dev, refs, settle=args.settle, settle_ms=args.settle_ms)
        log(f"other workloads: {json.dumps(other)}")

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    rec = dict(
        metric=METRIC, value=round(value, 1), unit="stamps/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, settle_steps=settle_steps, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="dev8-64x64-moffat-100k", n_stamps=args.n, W=W, K=8,
                    mixture="DEV8 synthetic (Dirichlet amplitudes, variances logspace 1e-4..10 r_e^2)",
                    psf="64x64 Moffat beta=3 FWHM 4.5 px + 1% Gaussian halo sigma 8 px",
                    routing="hybrid (smoothstep ramp n in [3,4])",
                    mean_K_F=round(float(kf.mean()), 3), mean_K_R=round(float(kr.mean()), 3)),
        roofline=roofline, cpu_baseline=cpu, parity=parity, rate_probes=probes,
        plain=plain, serving=serving, other_workloads=other, psf_cache_fill_ms=round(psf_cache_ms, 3),
        kernel_ms=dict(mean=round(avg_kern_ms, 4), median=round(float(np.median(kern_ms)), 4),
                       min=round(float(kern_ms.min()), 4), max=round(float(kern_ms.max()), 4)),
    )
    print(json.dumps(rec), flush=True)


def profile_set(gfc, ctx, dev, reps=3, settle=0):
    """Every kernel instantiation of the library, launched `reps` times after
    untimed launches (one, or with settle > 0 at least that many and 50 ms of
    device time), for rocprofv3 kernel traces and counters: the forward
    render at 16, 32, 64, 128 and 256 (the throughput workload's galaxies,
    radii scaled to the stamp; the large workload at 128 and 256), its
    eigen-PSF, Lanczos (fused at 64, separate passes at 128 and 256), Sersic
    and composite forms, the serving form with a per-galaxy PSF index, the
    adjoint at every size with the amplitude sums, and the PSF transforms.
    Returns the mean launch time of each case (HIP events)."""
    import torch

    d = lambda a: torch.as_tensor(a).to(dev)
    res = {}

    def run(name, n, fn):
        if settle > 0:
            settle_device(fn, settle, 50.0)
        else:
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = dict(stamps=n, ms=round(ms, 4), stamps_per_s=round(n / ms * 1e3, 1))
        log(f"profile set: {name}: {res[name]}")

    cfg = wl.config_metric()
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    rng = np.random.Generator(np.random.PCG64(8080))
    for W, n in ((16, 200_000), (32, 100_000), (64, 100_000), (128, 20_000)):
        g = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.5 * W / 64, 8.0 * W / 64))
        args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
        out = torch.empty((n, W, W), dtype=torch.float32, device=dev)
        psf.prepare(W)
        run(f"forward-{W}", n, lambda: gfc.gfc_render_stamps(ctx, psf, mix, *args, W, out=out))
        if W <= 128:
            run(f"lanczos-{W}", n, lambda: gfc.gfc_render_stamps(ctx, psf, mix, *args, W, out=out,
                                                                  flags=gfc.GFC_SHIFT_LANCZOS3))
        nb = min(n, 20_000)
        go = torch.randn((nb, W, W), device=dev, generator=torch.Generator(device=dev).manual_seed(W))
        ba = [a[:nb] for a in args]
        run(f"backward-{W}", nb, lambda: gfc.gfc_render_stamps_backward(ctx, psf, mix, *ba, W, go))
        del out, go
    c3 = wl.config3()
    g = c3["gal"].subset(np.nonzero(c3["gal"].W == 256)[0])
    psf3 = gfc.Psf(ctx, c3["psf"], c3.get("psf_gauss"))
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    out = torch.empty((len(g), 256, 256), dtype=torch.float32, device=dev)
    psf3.prepare(256)
    run("forward-256-large", len(g), lambda: gfc.gfc_render_stamps(ctx, psf3, mix, *args, 256, out=out))
    run("lanczos-256-large", len(g), lambda: gfc.gfc_render_stamps(ctx, psf3, mix, *args, 256, out=out,
                                                                  flags=gfc.GFC_SHIFT_LANCZOS3))
    del out
    nb = 2048
    go = torch.randn((nb, 256, 256), device=dev, generator=torch.Generator(device=dev).manual_seed(256))
    run("backward-256-large", nb, lambda: gfc.gfc_render_stamps_backward(ctx, psf3, mix, *[a[:nb] for a in args],
                                                                           256, go))
    del go
    psf3.close()
    # serving form: per-galaxy PSF index (requests of several PSFs fused), 64 x 64
    from paper_2012_15797_amd.serving import Server
    tr = wl.config4_trace(duration_s=0.05, rate_hz=2000.0, n_psf=8, restricted=False)
    psfs = [gfc.Psf(ctx, p) for p in tr["psfs"][:8]]
    tmix = gfc.Mixture.from_workload(ctx, tr["mix"].as_f32())
    srv = Server(ctx, mem_budget_bytes=8 << 30, n_streams=1, max_batch_stamps=1 << 20)
    g = wl.draw_galaxies(rng, 4096, 64, 0)

    def served():
        tk = [srv.submit(psfs[i % 8], tmix, 64, g.x[i::8], g.y[i::8], g.flux[i::8], g.r_e[i::8], g.e1[i::8],
                         g.e2[i::8]) for i in range(8)]
        for t in tk:
            srv.wait(t)
            srv.release(t)
    run("serving-64-8psf", len(g), served)
    srv.close()
    for p in psfs:
        p.close()
    tmix.close()
    # eigen-PSF, Sersic and composite forms at 64
    ce = wl.config_eigen()
    g, e = ce["gal"], ce["eig"]
    epsf = gfc.Psf.eigen(ctx, e["comps"], e["coef"], e["degree"], e["norm"])
    emix = gfc.Mixture.from_workload(ctx, ce["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    px, py = d(ce["psf_x"]), d(ce["psf_y"])
    out = torch.empty((len(g), 64, 64), dtype=torch.float32, device=dev)
    run("eigen-64", len(g), lambda: gfc.gfc_render_stamps(ctx, epsf, emix, *args, 64, out=out, psf_x=px, psf_y=py))
    epsf.close()
    emix.close()
    cs = wl.config_sersic()
    g = cs["gal"]
    fam = gfc.SersicFamily.from_workload(ctx, cs["family"])
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    sn = d(cs["sersic_n"])
    run("sersic-64", len(g), lambda: gfc.gfc_render_stamps_sersic(ctx, psf, fam, *args, sn, 64, out=out))
    fam.close()
    cc = wl.config_composite()
    g = cc["gal"]
    cmix = gfc.Mixture.from_workload(ctx, cc["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    fr, rh = d(cc["bulge_frac"]), d(cc["bulge_rho"])
    run("composite-64", len(g), lambda: gfc.gfc_render_stamps_composite(ctx, psf, cmix, 0, 1, *args, fr, rh, 64,
                                                                         out=out))
    cmix.close()
    del out
    # the PSF transforms (cold path): a fresh PSF per launch, every size
    P = cfg["psf"]

    def transforms():
        q = gfc.Psf(ctx, P)
        for W in (16, 32, 64, 128, 256):
            q.prepare(W)
        q.close()
    run("psf-transforms", 5, transforms)
    psf.close()
    mix.close()
    return res


def parity_of_rows(out, refs, dev):
    """Parity of the rows of `out` for which the CPU leg holds oracle stamps."""
    import torch

    if not refs:
        return None
    idx = sorted(refs)
    rows = out[torch.as_tensor(idx, device=dev)].cpu().numpy().astype(np.float64)
    return stamp_parity(rows, [refs[i] for i in idx])


def serving_benchmark(gfc, ctx, seconds, refs):
    """Open-loop replays of Poisson request traces against the
    continuous-batching server and against the plain mode (one launch per
    request, FIFO on one stream), with the same 32 GB device-memory budget:
    the full serving configuration (2,000 requests/s for `seconds`, 64
    resident PSFs, stamps 16..256), and the 64x64 one-PSF variant at the
    nominal and a saturating rate.  Each replay keeps the stamps of a seeded
    sample of its requests, checked against the CPU leg's oracle."""
    import torch

    from paper_2012_15797_amd.serving import Server, replay_trace

    out = {}
    for label, rate, secs, restricted in serving_traces(seconds):
        t0 = time.perf_counter()
        tr = wl.config4_trace(duration_s=secs, rate_hz=rate, restricted=restricted)
        log(f"serving trace {label or 'full_'}: {len(tr['requests'])} requests drawn in "
            f"{time.perf_counter() - t0:.1f} s")
        psfs = [gfc.Psf(ctx, p) for p in tr["psfs"]]
        mix = gfc.Mixture.from_workload(ctx, tr["mix"].as_f32())
        for p in psfs:
            for W in sorted({r["W"] for r in tr["requests"]}):
                p.prepare(W)
        what = ("64x64, DEV8, one PSF" if restricted else
                "stamp sizes 16..256, EXP6/DEV8, 64 PSFs")
        out[label + "trace"] = (f"{len(tr['requests'])} requests over {secs:.1f} s, Poisson {rate:.0f}/s, "
                                f"1..4096 galaxies log-uniform, {what}, budget 32 GB")
        sample = serving_sample(tr["requests"])
        ref = refs.get(f"serving_{label or 'full_'}")
        for name, streams, max_batch in (("batched", 2, 1 << 16), ("plain", 1, 0)):
            keep = {ri: torch.empty((len(tr["requests"][ri]["gal"]), tr["requests"][ri]["W"], tr["requests"][ri]["W"]),
                                    dtype=torch.float32, device=ctx.torch_device) for ri, _ in sample}
            srv = Server(ctx, mem_budget_bytes=32 << 30, n_streams=streams, max_batch_stamps=max_batch)
            out[label + name] = replay_trace(srv, tr["requests"], psfs, mix, keep=keep)
            srv.close()
            if ref is not None:
                rows = [keep[ri][gi].cpu().numpy().astype(np.float64) for ri, gis in sample for gi in gis]
                out[label + name]["parity"] = stamp_parity(rows, ref)
            del keep
            log(f"serving {label or 'full_'}{name}: {out[label + name]}")
        for p in psfs:
            p.close()
        mix.close()
    return out


def size_throughput(gfc, ctx, dev, refs, reps=5, settle=45, settle_ms=50.0):
    """Forward stamps/s per stamp size on the mixed-size and large-galaxy
    workloads (one launch per size bin), the 64x64 workload with Lanczos
    shifting, general Sersic, composites and the eigen-PSF, and the adjoint
    on the differentiation workload.  Every line carries the parity of a
    seeded sample of its own last launch against the CPU leg's oracle.
    Each case is timed after untimed launches of its own (at least `settle`
    launches and `settle_ms` of device time): the host work between cases
    idles the device, and the first tens of milliseconds of load after that
    run through the power-management transient the metric's settle steps
    skip."""
    import torch

    d = lambda a: torch.as_tensor(a).to(dev)

    def timed(fn, n_reps):
        settle_device(fn, max(3, settle), settle_ms)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n_reps

    def line(n, ms, **kw):
        return dict(stamps=n, ms=round(ms, 4), stamps_per_s=round(n / ms * 1e3, 1), **kw)

    def rows_parity(job, out_rows_of):
        """Parity of the job's reference sample; out_rows_of(global indices) -> rows."""
        if job not in refs:
            return None
        ii, ref = refs[job]
        return stamp_parity(out_rows_of(ii), ref)

    res = {}
    for cname, job, cfg in (("mixed-32-64-128", "mixed", wl.config2()), ("large-128-256", "large", wl.config3())):
        psf = gfc.Psf(ctx, cfg["psf"], cfg.get("psf_gauss"))
        mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
        g = cfg["gal"]
        tot_ms, tot_n = 0.0, 0
        worst = []
        for W in sorted(set(int(w) for w in g.W)):
            sel = np.nonzero(g.W == W)[0]
            sub = g.subset(sel)
            args = [d(a) for a in (sub.x, sub.y, sub.flux, sub.r_e, sub.e1, sub.e2)]
            mid = d(sub.mix_id)
            out = torch.empty((len(sub), W, W), dtype=torch.float32, device=dev)
            psf.prepare(W)
            ms = timed(lambda: gfc.gfc_render_stamps(ctx, psf, mix, *args, W, mix_id=mid, out=out), reps)
            par = None
            if job in refs:
                ii, ref = refs[job]
                keep = [(j, int(i)) for j, i in enumerate(ii) if g.W[i] == W]
                pos = np.searchsorted(sel, [i for _, i in keep])
                rows = out[torch.as_tensor(pos, device=dev)].cpu().numpy().astype(np.float64)
                par = stamp_parity(rows, [ref[j] for j, _ in keep])
                worst.append(par)
            res[f"{cname}/W{W}"] = line(len(sub), ms, parity=par,
                                        roofline=flops_roofline(workload_flops(sub, cfg["mix"], W), ms))
            tot_ms += ms
            tot_n += len(sub)
            del out
        par = None
        if worst:
            par = dict(n_checked=sum(p["n_checked"] for p in worst),
                       max_err_over_peak=max(p["max_err_over_peak"] for p in worst), tol=TOL_PEAK,
                       passed=all(p["passed"] for p in worst))
        res[cname] = line(tot_n, tot_ms, parity=par)
        psf.close()
        mix.close()

    # Lanczos-3 sub-pixel shift instead of the Fourier phase: the throughput workload
    cfg = wl.config_metric()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    out = torch.empty((len(g), 64, 64), dtype=torch.float32, device=dev)
    rows = lambda ii: out[torch.as_tensor(ii, device=dev)].cpu().numpy().astype(np.float64)
    ms = timed(lambda: gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, flags=gfc.GFC_SHIFT_LANCZOS3),
               reps * 4)
    res["lanczos3-dev8-64x64-100k"] = line(
        len(g), ms, parity=rows_parity("lanczos", rows),
        roofline=flops_roofline(workload_flops(g, cfg["mix"], 64) + len(g) * lanczos_flops(64), ms))
    psf.close()
    mix.close()

    # general Sersic (mixture interpolated per galaxy) and bulge + disk composites, 100k at 64x64
    cfg = wl.config_sersic()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    fam = gfc.SersicFamily.from_workload(ctx, cfg["family"])
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    sn = d(cfg["sersic_n"])
    ms = timed(lambda: gfc.gfc_render_stamps_sersic(ctx, psf, fam, *args, sn, 64, out=out), reps * 4)
    fam_t = cfg["family"]
    n_of = np.asarray(cfg["sersic_n"], np.float64)
    var_g = np.stack([np.interp(n_of, fam_t["n_grid"].astype(np.float64), fam_t["var"][:, k].astype(np.float64))
                      for k in range(fam_t["var"].shape[1])], axis=1)  # piecewise-linear in n, per component
    res["sersic8-64x64-100k"] = line(len(g), ms, parity=rows_parity("sersic", rows),
                                     roofline=flops_roofline(pergal_flops(g, var_g, 64), ms))
    psf.close()
    fam.close()
    cfg = wl.config_composite()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    fr, rh = d(cfg["bulge_frac"]), d(cfg["bulge_rho"])
    ms = timed(lambda: gfc.gfc_render_stamps_composite(ctx, psf, mix, 0, 1, *args, fr, rh, 64, out=out), reps * 4)
    _, var_d = cfg["mix"].table(0)
    _, var_b = cfg["mix"].table(1)
    rho2 = np.asarray(cfg["bulge_rho"], np.float64) ** 2
    var_g = np.concatenate([np.broadcast_to(var_d, (len(g), len(var_d))), rho2[:, None] * var_b[None, :]], axis=1)
    res["composite14-64x64-100k"] = line(len(g), ms, parity=rows_parity("composite", rows),
                                         roofline=flops_roofline(pergal_flops(g, var_g, 64), ms))
    psf.close()
    mix.close()

    # spatially varying PSF: 6 eigen components (degree-2 polynomial), 100k stamps at 64x64
    cfg = wl.config_eigen()
    g, e = cfg["gal"], cfg["eig"]
    psf = gfc.Psf.eigen(ctx, e["comps"], e["coef"], e["degree"], e["norm"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    px, py = d(cfg["psf_x"]), d(cfg["psf_y"])
    ms = timed(lambda: gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, psf_x=px, psf_y=py), reps * 4)
    J = len(e["comps"])
    res["eigenpsf6-dev8-64x64-100k"] = line(
        len(g), ms, parity=rows_parity("eigen", rows),
        roofline=flops_roofline(workload_flops(g, cfg["mix"], 64) + len(g) * eigen_psf_flops(64, J), ms))
    del out
    psf.close()
    mix.close()

    # adjoint on the differentiation workload (upstream gradient: seeded unit-normal noise)
    cfg = wl.config5()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    go = d(wl.generate.noise_field(BWD_NOISE_SEED, len(g), 64))
    ws = torch.empty(gfc.gfc_backward_workspace_bytes(len(g)) // 4 + 1, dtype=torch.float32, device=dev)
    gp = torch.empty((len(g), 6), dtype=torch.float32, device=dev)
    ga = torch.zeros((1, 16), dtype=torch.float32, device=dev)
    ms = timed(lambda: gfc.gfc_render_stamps_backward(ctx, psf, mix, *args, 64, go, grad_params=gp, grad_amp=ga,
                                                      workspace=ws), reps)
    par = None
    if "backward" in refs:
        ii, ref = refs["backward"]
        got = gp[torch.as_tensor(ii, device=dev)].cpu().numpy().astype(np.float64)
        ref = np.stack(ref)
        rms = np.sqrt(np.mean(ref**2, axis=0, keepdims=True))
        big = np.abs(ref) >= 1e-2 * rms
        bound = 1e-4 * np.abs(ref) + np.where(big, 0.0, 1e-5 * rms)
        rel = np.where(big, np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300), 0.0)
        par = dict(n_checked=int(len(ii)), max_rel_err=float(rel.max()), max_err_over_bound=float(
            (np.abs(got - ref) / bound).max()), tol="1e-4 relative where |oracle| >= 1e-2 rms, else + 1e-5 rms",
                   passed=bool((np.abs(got - ref) <= bound).all()))
    # The roofline takes the adjoint kernel's own time, as the headline's does:
    # the same call without an amplitude gradient launches that kernel alone
    # (it writes the same per-galaxy amplitude partials either way).
    ms_k = timed(lambda: gfc.gfc_render_stamps_backward(ctx, psf, mix, *args, 64, go, grad_params=gp, workspace=ws,
                                                        amp_grad=False), reps)
    fl = workload_flops(g, cfg["mix"], 64, adjoint=True)
    rl = flops_roofline(fl, ms_k)
    rl.update(kernel="render_bwd_small_kernel<64>", kernel_ms=round(ms_k, 4),
              frac_whole_call=flops_roofline(fl, ms)["frac"],
              note="achieved over the adjoint kernel's launch alone; frac_whole_call over the whole call, "
                   "amplitude-gradient reduction included")
    res["backward-dev8-64x64-10k"] = line(len(g), ms, parity=par, roofline=rl)
    psf.close()
    mix.close()
    return res


def plain_per_request(gfc, ctx, psf, mix, gal, W, dev, refs, seed=77):
    """The plain alternative to one batched launch: the same stamps split into
    requests of log-uniform 1..4096 galaxies, each with its own host-to-device
    parameter copy and its own launch, FIFO on one stream.  Parity: the
    stamps of the CPU leg's sample, from this run's output."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(gal)
    sizes = []
    tot = 0
    while tot < n:
        s = int(min(n - tot, max(1, math.floor(math.exp(rng.uniform(0, math.log(4097)))))))
        sizes.append(s)
        tot += s
    host = torch.from_numpy(np.stack([gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2])).pin_memory()
    dparams = torch.empty((6, n), dtype=torch.float32, device=dev)
    out = torch.empty((n, W, W), dtype=torch.float32, device=dev)

    def run():
        off = 0
        for s in sizes:
            dparams[:, off:off + s].copy_(host[:, off:off + s], non_blocking=True)
            p = dparams[:, off:off + s]
            gfc.gfc_render_stamps(ctx, psf, mix, p[0], p[1], p[2], p[3], p[4], p[5], W,
                                  out=out[off:off + s])
            off += s

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(value=round(n / dt, 1), unit="stamps/s", requests=len(sizes),
                mean_request=round(n / len(sizes), 1), parity=parity_of_rows(out, refs, dev),
                note="one launch per request incl. its H2D parameter copy, FIFO on one stream")


if __name__ == "__main__":
    main()
