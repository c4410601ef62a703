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

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""

from __future__ import annotations

import argparse
import json
import math
import os
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
HBM_GBPS = 8000.0

KQ = -2.0 * math.pi**2 * math.log2(math.e)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- work accounting
def routing_counts(gal, var, W):
    """K_F (components with Fourier weight > 0) and K_R (weight < 1) per galaxy,
    from the closed-form pixel covariance trace: tr C_i = v_i r_e^2 (2 + 2 e^2)/(1 + e)^2."""
    r = gal.r_e.astype(np.float64)
    e = np.hypot(gal.e1.astype(np.float64), gal.e2.astype(np.float64))
    tr = r * r * (2.0 + 2.0 * e * e) / (1.0 + e) ** 2
    n = (W / 2.0) / np.sqrt(var[None, :] * tr[:, None])
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


# ---------------------------------------------------------------- CPU baseline (oracle)
def _oracle_worker(args):
    idx, seed_n = args
    import threadpoolctl

    import oracle as o

    with threadpoolctl.threadpool_limits(1):
        cfg = wl.config_metric(seed_n)
        P = cfg["psf"].astype(np.float64)
        t0 = time.perf_counter()
        imgs = o.render_batch(P, cfg["mix"].as_f32(), cfg["gal"], idx=idx)
        dt = time.perf_counter() - t0
    return idx, np.stack(imgs), dt


def cpu_baseline(n_total, sample, workers):
    """Times the FP64 oracle (unchanged) on a seeded sample of the workload,
    one single-threaded process per core.  Runs before the GPU is touched."""
    import multiprocessing as mp

    rng = np.random.Generator(np.random.PCG64(2024))
    idx = np.sort(rng.choice(n_total, size=sample, replace=False))
    chunks = [(list(map(int, c)), n_total) for c in np.array_split(idx, workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, chunks)
    wall = time.perf_counter() - t0
    stamps = {}
    cpu_s = 0.0
    for ii, imgs, dt in res:
        cpu_s += dt
        for j, i in enumerate(ii):
            stamps[i] = imgs[j]
    return dict(value=sample / wall, unit="stamps/s", cores=workers, kind="oracle",
                sample=f"{sample} seeded stamps of the 100k workload, FP64 oracle, {workers} "
                       f"single-threaded processes, {cpu_s:.1f} CPU-s in {wall:.2f} s wall"), stamps


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--cpu-sample", type=int, default=24000)
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="length of the Poisson request trace replayed against the server (0: skip)")
    ap.add_argument("--no-other", action="store_true", help="skip the other-workload throughput table")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this renderer runs on one GPU; --gpus must be 1 "
              "(stamps are independent, so more GPUs would each take a shard of the batch)",
              file=sys.stderr)
        sys.exit(2)

    cfg = wl.config_metric(args.n)
    gal = cfg["gal"]
    W = 64
    mixf = cfg["mix"].as_f32()
    amp, var = mixf.table(0)
    kf, kr = routing_counts(gal, var, W)
    flops_stamp = algorithmic_flops_per_stamp(W, kf, kr)

    cpu, oracle_stamps = None, {}
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        log(f"cpu baseline: oracle on {args.cpu_sample} stamps with {workers} processes")
        cpu, oracle_stamps = cpu_baseline(args.n, args.cpu_sample, workers)
        log(f"cpu baseline: {cpu['value']:.1f} stamps/s")

    import torch

    import paper_2012_15797_amd as gfc

    dev = torch.device("cuda", 0)
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    stream = torch.cuda.current_stream(dev)
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
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall_s * 1e3 / args.steps
    value = args.n / (ms_per_step / 1e3)
    avg_kern_ms = float(np.mean(kern_ms))
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, kernel {avg_kern_ms:.3f} ms avg "
        f"(min {min(kern_ms):.3f})")

    achieved_tflops = float(flops_stamp.sum()) / (avg_kern_ms * 1e-3) / 1e12
    roofline = dict(bound="alu", achieved=round(achieved_tflops, 3), peak=round(FP32_FMA_NONPACKED_TFLOPS, 2),
                    unit="TFLOP/s", frac=round(achieved_tflops / FP32_FMA_NONPACKED_TFLOPS, 4), traffic=measured_traffic(),
                    kernel="render_small_kernel<64, false, false>",
                    flops_per_stamp=round(float(flops_stamp.mean()), 1),
                    algorithmic_bytes=args.n * (4 * W * W + 28),
                    hbm_gbps=round(args.n * (4 * W * W + 28) / (avg_kern_ms * 1e-3) / 1e9, 1))

    parity = None
    if oracle_stamps:
        idx = sorted(oracle_stamps)
        sel = out[torch.as_tensor(idx, device=dev)].cpu().numpy().astype(np.float64)
        errs = [np.abs(sel[j] - oracle_stamps[i]).max() / np.abs(oracle_stamps[i]).max()
                for j, i in enumerate(idx)]
        parity = dict(n_checked=len(idx), max_err_over_peak=float(max(errs)), tol=1e-5,
                      passed=bool(max(errs) <= 1e-5))
        log(f"parity on {len(idx)} stamps: max err/peak {max(errs):.2e}")

    plain = None
    if not args.no_plain:
        plain = plain_per_request(gfc, ctx, psf, mix, gal, W, dev)
        log(f"plain per-request launches: {plain['value']:.3e} stamps/s over {plain['requests']} requests")

    serving = None
    if args.serve_seconds > 0:
        serving = serving_benchmark(gfc, ctx, args.serve_seconds)

    other = None
    if not args.no_other:
        other = size_throughput(gfc, ctx, dev)
        log(f"other workloads: {other}")

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
        warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="dev8-64x64-moffat-100k", n_stamps=args.n, W=W, K=8,
                    mixture="DEV8 synthetic (Dirichlet amplitudes, variances logspace 1e-4..10 r_e^2)",
                    psf="64x64 Moffat beta=3 FWHM 4.5 px + 1% Gaussian halo sigma 8 px",
                    routing="hybrid (smoothstep ramp n in [3,4])",
                    mean_K_F=round(float(kf.mean()), 3), mean_K_R=round(float(kr.mean()), 3)),
        roofline=roofline, cpu_baseline=cpu, parity=parity,
        plain=plain, serving=serving, other_workloads=other, psf_cache_fill_ms=round(psf_cache_ms, 3),
        kernel_ms=dict(mean=round(avg_kern_ms, 4), min=round(min(kern_ms), 4), max=round(max(kern_ms), 4)),
    )
    print(json.dumps(rec), flush=True)


def serving_benchmark(gfc, ctx, seconds):
    """Open-loop replay of the 64x64 serving trace (Poisson arrivals at
    2,000 requests/s, 1..4096 galaxies per request, DEV8, the throughput
    workload's PSF) against the continuous-batching server and against the
    plain mode (one launch per request, FIFO on one stream), with the same
    32 GB device-memory budget."""
    from paper_2012_15797_amd.serving import Server, replay_trace

    out = {}
    for label, rate, secs, restricted in (("", 2000.0, seconds, True),
                                          ("saturated_", 20000.0, min(seconds, 1.0), True),
                                          ("mixed_sizes_", 2000.0, min(seconds, 1.0), False)):
        tr = wl.config4_trace(duration_s=secs, rate_hz=rate, restricted=restricted)
        psfs = [gfc.Psf(ctx, p) for p in tr["psfs"]]
        mix = gfc.Mixture.from_workload(ctx, tr["mix"].as_f32())
        for p in psfs:
            for W in sorted({r["W"] for r in tr["requests"]}):
                p.prepare(W)
        what = ("64x64, DEV8, one PSF" if restricted else
                "stamp sizes 16..256, EXP6/DEV8, 64 PSFs")
        out[label + "trace"] = (f"{len(tr['requests'])} requests over {secs:.1f} s, Poisson {rate:.0f}/s, "
                                f"1..4096 galaxies log-uniform, {what}, budget 32 GB")
        for name, streams, max_batch in (("batched", 2, 1 << 16), ("plain", 1, 0)):
            srv = Server(ctx, mem_budget_bytes=32 << 30, n_streams=streams, max_batch_stamps=max_batch)
            out[label + name] = replay_trace(srv, tr["requests"], psfs, mix)
            srv.close()
            log(f"serving {label or 'nominal_'}{name}: {out[label + name]}")
        for p in psfs:
            p.close()
        mix.close()
    return out


def size_throughput(gfc, ctx, dev, reps=5):
    """Forward stamps/s per stamp size on the mixed-size and large-galaxy
    workloads (one launch per size bin), and the adjoint on the
    differentiation workload."""
    import torch

    res = {}
    for cname, cfg in (("mixed-32-64-128", wl.config2()), ("large-128-256", wl.config3())):
        psf = gfc.Psf(ctx, cfg["psf"], cfg.get("psf_gauss"))
        mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
        g = cfg["gal"]
        tot_ms, tot_n = 0.0, 0
        for W in sorted(set(int(w) for w in g.W)):
            sub = g.subset(np.nonzero(g.W == W)[0])
            d = lambda a: torch.as_tensor(a).to(dev)
            args = [d(a) for a in (sub.x, sub.y, sub.flux, sub.r_e, sub.e1, sub.e2)]
            mid = d(sub.mix_id)
            out = torch.empty((len(sub), W, W), dtype=torch.float32, device=dev)
            psf.prepare(W)
            gfc.gfc_render_stamps(ctx, psf, mix, *args, W, mix_id=mid, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                gfc.gfc_render_stamps(ctx, psf, mix, *args, W, mix_id=mid, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[f"{cname}/W{W}"] = dict(stamps=len(sub), ms=round(ms, 4), stamps_per_s=round(len(sub) / ms * 1e3, 1))
            tot_ms += ms
            tot_n += len(sub)
            del out
        res[cname] = dict(stamps=tot_n, ms=round(tot_ms, 4), stamps_per_s=round(tot_n / tot_ms * 1e3, 1))
        psf.close()
        mix.close()
    # Lanczos-3 sub-pixel shift instead of the Fourier phase: the throughput workload
    cfg = wl.config_metric()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    d = lambda a: torch.as_tensor(a).to(dev)
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    out = torch.empty((len(g), 64, 64), dtype=torch.float32, device=dev)
    for _ in range(3):
        gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, flags=gfc.GFC_SHIFT_LANCZOS3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps * 4):
        gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, flags=gfc.GFC_SHIFT_LANCZOS3)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (reps * 4)
    res["lanczos3-dev8-64x64-100k"] = dict(stamps=len(g), ms=round(ms, 4), stamps_per_s=round(len(g) / ms * 1e3, 1))
    del out
    psf.close()
    mix.close()
    # general Sersic (mixture interpolated per galaxy) and bulge + disk composites, 100k at 64x64
    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps * 4):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (reps * 4)

    cfg = wl.config_sersic()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    fam = gfc.SersicFamily.from_workload(ctx, cfg["family"])
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    sn = d(cfg["sersic_n"])
    out = torch.empty((len(g), 64, 64), dtype=torch.float32, device=dev)
    ms = timed(lambda: gfc.gfc_render_stamps_sersic(ctx, psf, fam, *args, sn, 64, out=out))
    res["sersic8-64x64-100k"] = dict(stamps=len(g), ms=round(ms, 4), stamps_per_s=round(len(g) / ms * 1e3, 1))
    psf.close()
    fam.close()
    cfg = wl.config_composite()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    fr, rh = d(cfg["bulge_frac"]), d(cfg["bulge_rho"])
    ms = timed(lambda: gfc.gfc_render_stamps_composite(ctx, psf, mix, 0, 1, *args, fr, rh, 64, out=out))
    res["composite14-64x64-100k"] = dict(stamps=len(g), ms=round(ms, 4), stamps_per_s=round(len(g) / ms * 1e3, 1))
    del out
    psf.close()
    mix.close()
    # spatially varying PSF: 6 eigen components (degree-2 polynomial), 100k stamps at 64x64
    cfg = wl.config_eigen()
    g, e = cfg["gal"], cfg["eig"]
    psf = gfc.Psf.eigen(ctx, e["comps"], e["coef"], e["degree"], e["norm"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    d = lambda a: torch.as_tensor(a).to(dev)
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    px, py = d(cfg["psf_x"]), d(cfg["psf_y"])
    out = torch.empty((len(g), 64, 64), dtype=torch.float32, device=dev)
    for _ in range(3):
        gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, psf_x=px, psf_y=py)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps * 4):
        gfc.gfc_render_stamps(ctx, psf, mix, *args, 64, out=out, psf_x=px, psf_y=py)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (reps * 4)
    res["eigenpsf6-dev8-64x64-100k"] = dict(stamps=len(g), ms=round(ms, 4), stamps_per_s=round(len(g) / ms * 1e3, 1))
    del out
    psf.close()
    mix.close()
    # adjoint on the differentiation workload (upstream gradient: unit normal noise)
    cfg = wl.config5()
    g = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    d = lambda a: torch.as_tensor(a).to(dev)
    args = [d(a) for a in (g.x, g.y, g.flux, g.r_e, g.e1, g.e2)]
    go = torch.randn((len(g), 64, 64), device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    ws = torch.empty(gfc.gfc_backward_workspace_bytes(len(g)) // 4 + 1, dtype=torch.float32, device=dev)
    gp = torch.empty((len(g), 6), dtype=torch.float32, device=dev)
    ga = torch.zeros((1, 16), dtype=torch.float32, device=dev)
    gfc.gfc_render_stamps_backward(ctx, psf, mix, *args, 64, go, grad_params=gp, grad_amp=ga, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gfc.gfc_render_stamps_backward(ctx, psf, mix, *args, 64, go, grad_params=gp, grad_amp=ga, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res["backward-dev8-64x64-10k"] = dict(stamps=len(g), ms=round(ms, 4), stamps_per_s=round(len(g) / ms * 1e3, 1))
    psf.close()
    mix.close()
    return res


def plain_per_request(gfc, ctx, psf, mix, gal, W, dev, seed=77):
    """The plain alternative to one batched launch: the same stamps split into
    requests of log-uniform 1..4096 galaxies, each with its own host-to-device
    parameter copy and its own launch, FIFO on one stream."""
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
                mean_request=round(n / len(sizes), 1),
                note="one launch per request incl. its H2D parameter copy, FIFO on one stream")


if __name__ == "__main__":
    main()
