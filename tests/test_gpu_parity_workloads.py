"""GPU parity on the full synthetic workloads, launched as the benchmark
launches them, checked on stratified samples against the FP64 oracle:

- mixed sizes: all 100,000 galaxies (32/64/128 in 5:4:1, two tables), one
  launch per stamp size; 2,000 stamps sampled across every (size, table,
  real-space component count) class;
- large galaxies: all 20,000 (128 and 256), one launch per size; 500 stamps
  sampled the same way;
- differentiation: 500 galaxies of the 10,000-galaxy fit workload with the
  fit's upstream gradient (I - T) / sigma^2.

Forward bar: per stamp, max |gpu - oracle| <= 1e-5 x max |oracle|; adjoint
bar: that of tests/gpu_helpers.py."""

import numpy as np
import pytest

import oracle as o
import workloads as wl
from gpu_helpers import TOL_PEAK, assert_grads_close, gpu_grads, lib_objects, oracle_grads, oracle_stamps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


def _real_space_counts(cfg, gal):
    """Number of components with a real-space share per galaxy (the class a
    stamp falls in for sampling only: n_i = (W/2)/sqrt(tr C_i) <= 4)."""
    m = cfg["mix"].as_f32()
    out = np.zeros(len(gal), np.int32)
    r = gal.r_e.astype(np.float64)
    e = np.hypot(gal.e1.astype(np.float64), gal.e2.astype(np.float64))
    tr0 = r * r * (2.0 + 2.0 * e * e) / (1.0 + e) ** 2
    for t in range(m.n_tables):
        sel = gal.mix_id == t
        _, var = m.table(t)
        n = (gal.W[sel, None] / 2.0) / np.sqrt(var[None, :] * tr0[sel, None])
        out[sel] = (n < 4.0).sum(axis=1)
    return out


def _stratified(classes, total, rng, floor=10):
    """Indices: every class gets min(size, floor), the rest proportionally."""
    keys, inv = np.unique(classes, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    pick = []
    sizes = np.bincount(inv, minlength=len(keys))
    quota = np.maximum(np.minimum(sizes, floor), np.round(total * sizes / sizes.sum()).astype(int))
    quota = np.minimum(quota, sizes)
    for c in range(len(keys)):
        members = np.nonzero(inv == c)[0]
        pick.extend(rng.choice(members, quota[c], replace=False).tolist())
    return np.array(sorted(pick)), keys


def _render_by_size(ctx, cfg):
    """One launch per stamp size, into per-size output buffers (the benchmark's
    launch configuration).  Returns {W: (galaxy indices, output tensor)}."""
    import torch
    import paper_2012_15797_amd as gfc

    psf, mix = lib_objects(ctx, cfg)
    gal = cfg["gal"]
    out = {}
    for W in sorted(set(int(w) for w in gal.W)):
        sel = np.nonzero(gal.W == W)[0]
        sub = gal.subset(sel)
        out[W] = (sel, gfc.gfc_render_stamps(ctx, psf, mix, sub.x, sub.y, sub.flux, sub.r_e, sub.e1, sub.e2,
                                             W, mix_id=sub.mix_id))
    torch.cuda.synchronize()
    return psf, mix, out


def _check_sample(cfg, out, idx, label):
    import torch

    gal = cfg["gal"]
    worst = 0.0
    per_w = {}
    for W, (sel, t) in out.items():
        pos = np.searchsorted(sel, idx[np.isin(idx, sel)])
        if len(pos) == 0:
            continue
        rows = t[torch.as_tensor(pos, device=t.device)].cpu().numpy().astype(np.float64)
        gidx = sel[pos]
        ref = oracle_stamps(cfg, gal, gidx)
        errs = np.array([np.abs(rows[j] - ref[j]).max() / np.abs(ref[j]).max() for j in range(len(gidx))])
        assert np.isfinite(rows).all()
        per_w[W] = (len(gidx), float(errs.max()))
        worst = max(worst, float(errs.max()))
        assert errs.max() <= TOL_PEAK, (label, W, float(errs.max()), int(gidx[errs.argmax()]))
    print(f"[parity] {label}: {len(idx)} stamps, worst err/peak {worst:.2e}, per size {per_w}")
    return per_w


def test_mixed_workload_stratified_2000(ctx):
    import torch

    cfg = wl.config2()
    gal = cfg["gal"]
    kr = _real_space_counts(cfg, gal)
    classes = np.stack([gal.W, gal.mix_id, np.minimum(kr, 4)], axis=1)
    idx, keys = _stratified(classes, 2000, np.random.Generator(np.random.PCG64(2001)))
    assert len(idx) >= 2000
    psf, mix, out = _render_by_size(ctx, cfg)
    for W, (sel, t) in out.items():
        assert bool(torch.isfinite(t).all()), W
    per_w = _check_sample(cfg, out, idx, "mixed 32/64/128 workload")
    assert set(per_w) == {32, 64, 128}
    del out
    psf.close(); mix.close()


def test_large_workload_stratified_500(ctx):
    import torch

    cfg = wl.config3()
    gal = cfg["gal"]
    kr = _real_space_counts(cfg, gal)
    classes = np.stack([gal.W, np.minimum(kr, 4)], axis=1)
    idx, keys = _stratified(classes, 500, np.random.Generator(np.random.PCG64(2002)))
    assert len(idx) >= 500
    psf, mix, out = _render_by_size(ctx, cfg)
    for W, (sel, t) in out.items():
        assert bool(torch.isfinite(t).all()), W
    per_w = _check_sample(cfg, out, idx, "large 128/256 workload")
    assert set(per_w) == {128, 256}
    del out
    psf.close(); mix.close()


def test_fit_workload_adjoint_500(ctx):
    """The differentiation workload's upstream gradient (I - T) / sigma^2,
    T = render at perturbed parameters plus noise of 0.01 x peak, on 500
    galaxies spread over the 10,000."""
    cfg = wl.config5()
    idx = np.random.Generator(np.random.PCG64(2003)).choice(len(cfg["gal"]), 500, replace=False)
    idx.sort()
    gal, tgt = cfg["gal"].subset(idx), cfg["target_gal"].subset(idx)
    P = cfg["psf"].astype(np.float64)
    I = np.stack(o.render_batch(P, cfg["mix"].as_f32(), gal))
    T = np.stack(o.render_batch(P, cfg["mix"].as_f32(), tgt))
    peak = np.abs(T).max(axis=(1, 2), keepdims=True)
    sigma = 0.01 * peak
    noise = wl.generate.noise_field(cfg["noise_seed"], len(cfg["gal"]), 64)[idx]
    g = ((I - (T + sigma * noise)) / sigma**2).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, 64, g)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g)
    assert_grads_close(gp, rp, "params fit workload, 500 galaxies")
    assert_grads_close(ga, ra, "amplitudes fit workload, 500 galaxies", scale=ra_abs)
    psf.close(); mix.close()
