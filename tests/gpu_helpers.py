"""Helpers shared by the GPU parity tests: build library objects from a
workload and compare stamps with the FP64 oracle."""

import numpy as np

import oracle as o

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
