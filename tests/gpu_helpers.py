"""Helpers shared by the GPU parity tests: build library objects from a
workload and compare stamps and gradients with the FP64 oracle."""

import numpy as np

import oracle as o
from oracle.grad import PARAMS

# Forward parity bar: per stamp, max |gpu - oracle| <= TOL_PEAK * max |oracle|.
TOL_PEAK = 1e-5


def lib_objects(ctx, cfg, psf_gauss=None):
    import paper_2012_15797_amd as gfc

    gauss = cfg.get("psf_gauss") if psf_gauss is None else psf_gauss
    psf = gfc.Psf(ctx, cfg["psf"], gauss)
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    return psf, mix


def render_gpu(ctx, psf, mix, gal, W, flags=0, cd=None):
    import paper_2012_15797_amd as gfc
    import torch

    out = gfc.gfc_render_stamps(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W,
                                mix_id=gal.mix_id, flags=flags, cd=cd)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def oracle_stamps(cfg, gal, idx, flags=0, cd=None, gauss=None):
    """Oracle stamps from the same float32 inputs the GPU received."""
    P = np.asarray(cfg["psf"], np.float32).astype(np.float64) if cfg["psf"].dtype == np.float32 \
        else np.asarray(cfg["psf"], np.float64)
    g = gauss if gauss is not None else cfg.get("psf_gauss")
    return o.render_batch(P, cfg["mix"].as_f32(), gal, flags=flags, psf_gauss=g, cd=cd, idx=idx)


def peak_errors(gpu, ref_list, idx):
    errs = []
    for j, i in enumerate(idx):
        ref = ref_list[j]
        peak = np.abs(ref).max()
        errs.append(np.abs(gpu[i] - ref).max() / peak)
    return np.array(errs)


# Adjoint parity bar: per parameter, |gpu - oracle| <= GRAD_RTOL |oracle| where
# |oracle| >= GRAD_REL_FLOOR x scale; below that GRAD_ATOL_RMS x scale is
# added, since the float32 rounding of a result that cancels is set by the
# size of the summed terms, not by the result.  For per-galaxy gradients the
# scale is the rms over the case's galaxies (a galaxy far fainter than the
# brightest, or a derivative that cancels against its own terms); for the
# per-table amplitude sums it is the sum of the absolute per-galaxy
# contributions (galaxies whose contributions cancel in the table's sum).
GRAD_RTOL, GRAD_ATOL_RMS, GRAD_REL_FLOOR = 1e-4, 1e-5, 1e-2


def oracle_grads(cfg, gal, g, flags=0, cd=None, gauss=None, mix=None, psf=None):
    """Per-galaxy dL/d(x, y, flux, log r_e, e1, e2), per-table amplitude sums
    [n_tables][16] and the sums of their absolute per-galaxy terms, from the
    FP64 analytic Jacobian with the float32 inputs the GPU saw."""
    mix = cfg["mix"].as_f32() if mix is None else mix
    P = np.asarray(cfg["psf"] if psf is None else psf, np.float32).astype(np.float64)
    if gauss is None:
        gauss = cfg.get("psf_gauss")
    gauss = o.psf_gauss_moments(P) if gauss is None else np.asarray(gauss, np.float64)
    cache = {}
    gp = np.zeros((len(gal), 6))
    ga = np.zeros((mix.n_tables, 16))
    ga_abs = np.zeros((mix.n_tables, 16))
    for i in range(len(gal)):
        p = gal.params(i)
        W = p["W"]
        if W not in cache:
            cache[W] = o.psf_spectrum(P, W)
        amp, var = mix.table(p["mix_id"])
        _, J = o.render_stamp_jacobian(cache[W], gauss, amp, var, p["x"], p["y"], p["flux"], p["r_e"],
                                       p["e1"], p["e2"], W, flags, cd)
        lg = o.loss_gradient(np.asarray(g[i], np.float64), J)
        gp[i] = [lg[k] for k in PARAMS]
        ga[p["mix_id"], : len(amp)] += lg["amp"]
        ga_abs[p["mix_id"], : len(amp)] += np.abs(lg["amp"])
    return gp, ga, ga_abs


def gpu_grads(ctx, psf, mix, gal, W, g, flags=0, cd=None):
    import torch
    import paper_2012_15797_amd as gfc

    gt = torch.as_tensor(np.ascontiguousarray(g, np.float32)).cuda()
    gp, ga = gfc.gfc_render_stamps_backward(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1,
                                            gal.e2, W, gt, mix_id=gal.mix_id, flags=flags, cd=cd)
    torch.cuda.synchronize()
    return gp.cpu().numpy().astype(np.float64), ga.cpu().numpy().astype(np.float64)


def grad_errors(gpu, ref, scale=None):
    """(bound array, worst pure relative error over the entries with
    |oracle| >= GRAD_REL_FLOOR x scale, number of such entries).  scale:
    None for the rms over axis 0, else an array like ref."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if scale is None:
        scale = np.sqrt(np.mean(ref**2, axis=0, keepdims=True))
    big = np.abs(ref) >= GRAD_REL_FLOOR * scale
    bound = GRAD_RTOL * np.abs(ref) + np.where(big, 0.0, GRAD_ATOL_RMS * scale)
    rel = np.where(big & (ref != 0), np.abs(gpu - ref) / np.where(ref != 0, np.abs(ref), 1.0), 0.0)
    return np.broadcast_to(bound, ref.shape), float(rel.max()) if rel.size else 0.0, int(big.sum())


def assert_grads_close(gpu, ref, what, scale=None):
    """The adjoint bar above; prints the worst pure relative error of the
    entries it applies to.  Returns that error.  Amplitude sums pass the
    oracle's sums of absolute terms as scale."""
    bound, worst_rel, n_rel = grad_errors(gpu, ref, scale)
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    bad = err > bound
    print(f"[grad parity] {what}: worst relative error {worst_rel:.2e} over {n_rel} entries "
          f"with |oracle| >= {GRAD_REL_FLOOR:g} of its scale; worst err/bound {float((err / np.maximum(bound, 1e-300)).max()):.3f}")
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        worst = float((err / np.maximum(bound, 1e-300)).max())
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} out of tolerance (worst {worst:.2f}x "
                             f"the bound); first {i}: gpu {gpu[i]:.6e} oracle {ref[i]:.6e} bound {bound[i]:.3e}")
    return worst_rel
