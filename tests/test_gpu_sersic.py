"""GPU parity of general-Sérsic (interpolated mixtures), composite
(bulge + disk) renders and stamp accumulation, through the C ABI, against the
FP64 oracle (oracle/sersic.py).  Bar: per stamp, max |gpu - oracle| <=
1e-5 x max |oracle|."""

import numpy as np
import pytest

import oracle as o
from oracle import sersic as osr
import workloads as wl
from gpu_helpers import TOL_PEAK

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _check(gpu, ref, idx):
    errs = np.array([np.abs(gpu[i] - r).max() / np.abs(r).max() for i, r in zip(idx, ref)])
    assert errs.max() <= TOL_PEAK, (errs.max(), int(np.argmax(errs)))


def _sersic(ctx, gal, sn, W, fam, P, flags=0):
    import paper_2012_15797_amd as gfc
    psf = gfc.Psf(ctx, P)
    f = gfc.SersicFamily.from_workload(ctx, fam)
    out = gfc.gfc_render_stamps_sersic(ctx, psf, f, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, sn, W,
                                       flags=flags)
    res = _np(out)
    psf.close(); f.close()
    return res


@pytest.mark.parametrize("W", [16, 32, 64, 128, 256])
def test_sersic_each_size(ctx, W):
    rng = np.random.Generator(np.random.PCG64(1000 + W))
    fam = wl.sersic_family()
    n = 40 if W < 256 else 8
    gal = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.3, W / 4.0))
    sn = rng.uniform(0.5, 6.0, n).astype(np.float32)
    sn[:3] = fam["n_grid"][[0, 5, -1]]  # grid nodes and both ends
    P = wl.psf_moffat_halo(64).astype(np.float32)
    gpu = _sersic(ctx, gal, sn, W, fam, P)
    idx = list(range(n))
    ref = osr.render_batch_sersic(P.astype(np.float64), fam, gal, sn, idx=idx)
    _check(gpu, ref, idx)


def test_sersic_off_grid_is_nan_and_counted(ctx):
    fam = wl.sersic_family()
    cfg = wl.config_metric(6)
    gal = cfg["gal"]
    sn = np.array([1.0, 0.4, 7.0, np.nan, 2.0, 6.0], np.float32)
    before = ctx.invalid_count()
    gpu = _sersic(ctx, gal, sn, 64, fam, cfg["psf"])
    assert ctx.invalid_count() - before == 3
    bad = np.isnan(gpu).all(axis=(1, 2))
    assert bad.tolist() == [False, True, True, True, False, False]


def test_full_size_sersic_sampled(ctx):
    cfg = wl.config_sersic()
    gal = cfg["gal"]
    gpu = _sersic(ctx, gal, cfg["sersic_n"], 64, cfg["family"], cfg["psf"])
    assert np.isfinite(gpu).all()
    rng = np.random.Generator(np.random.PCG64(1010))
    idx = sorted(set(rng.choice(len(gal), 100, replace=False).tolist()) | {0, len(gal) - 1})
    ref = osr.render_batch_sersic(cfg["psf"].astype(np.float64), cfg["family"], gal, cfg["sersic_n"], idx=idx)
    _check(gpu, ref, idx)


def _composite_oracle(cfg, gal, frac, rho, idx, flags=0):
    P = cfg["psf"].astype(np.float64)
    mix = cfg["mix"].as_f32()
    (ad, vd), (ab, vb) = mix.table(0), mix.table(1)
    cache, out = {}, []
    for i in idx:
        p = gal.params(int(i))
        W = p["W"]
        if W not in cache:
            cache[W] = o.psf_spectrum(P, W)
        a, v = osr.composite_mixture(ad, vd, ab, vb, float(frac[i]), float(rho[i]))
        out.append(o.render_stamp(cache[W], o.psf_gauss_moments(P), a, v, p["x"], p["y"], p["flux"], p["r_e"],
                                  p["e1"], p["e2"], W, flags))
    return out


@pytest.mark.parametrize("W", [16, 32, 64, 128, 256])
def test_composite_each_size(ctx, W):
    import paper_2012_15797_amd as gfc
    cfg = wl.config_composite(10)
    rng = np.random.Generator(np.random.PCG64(1020 + W))
    n = 30 if W < 256 else 6
    gal = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.5, W / 5.0))
    frac = rng.uniform(0, 1, n).astype(np.float32)
    frac[:2] = [0.0, 1.0]
    rho = np.exp(rng.uniform(np.log(0.2), 0.0, n)).astype(np.float32)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    out = gfc.gfc_render_stamps_composite(ctx, psf, mix, 0, 1, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2,
                                          frac, rho, W)
    gpu = _np(out)
    idx = list(range(n))
    _check(gpu, _composite_oracle(cfg, gal, frac, rho, idx), idx)
    psf.close(); mix.close()


def test_accumulate_two_shapes_in_one_stamp(ctx):
    """A disk and a bulge with different ellipticities and radii: two calls,
    the second with GFC_ACCUMULATE, equal the sum of the two oracle stamps."""
    import paper_2012_15797_amd as gfc
    cfg = wl.config_composite(10)
    rng = np.random.Generator(np.random.PCG64(1030))
    n = 20
    disk = wl.draw_galaxies(rng, n, 64, 0)
    bulge = wl.draw_galaxies(rng, n, 64, 1, r_e_range=(0.3, 3.0))
    bulge.x[:], bulge.y[:] = disk.x, disk.y
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    out = gfc.gfc_render_stamps(ctx, psf, mix, disk.x, disk.y, disk.flux, disk.r_e, disk.e1, disk.e2, 64,
                                mix_id=disk.mix_id)
    gfc.gfc_render_stamps(ctx, psf, mix, bulge.x, bulge.y, bulge.flux, bulge.r_e, bulge.e1, bulge.e2, 64,
                          mix_id=bulge.mix_id, flags=gfc.GFC_ACCUMULATE, out=out)
    gpu = _np(out)
    P = cfg["psf"].astype(np.float64)
    idx = list(range(n))
    ref_d = o.render_batch(P, cfg["mix"].as_f32(), disk, idx=idx)
    ref_b = o.render_batch(P, cfg["mix"].as_f32(), bulge, idx=idx)
    _check(gpu, [a + b for a, b in zip(ref_d, ref_b)], idx)
    with pytest.raises(gfc.GfcError) as e:
        gfc.gfc_render_stamps(ctx, psf, mix, disk.x, disk.y, disk.flux, disk.r_e, disk.e1, disk.e2, 64,
                              flags=gfc.GFC_ACCUMULATE | gfc.GFC_SHIFT_LANCZOS3, out=out)
    assert e.value.status == -1
    psf.close(); mix.close()


@pytest.mark.parametrize("W", [16, 128, 256])
def test_accumulate_each_size(ctx, W):
    """GFC_ACCUMULATE at the other stamp sizes (several stamps per wavefront,
    two wavefronts per stamp, the persistent 256 x 256 kernel): a second render
    into the same stamps adds to them."""
    import paper_2012_15797_amd as gfc
    cfg = wl.config_composite(10)
    rng = np.random.Generator(np.random.PCG64(1050 + W))
    n = 12 if W < 256 else 4
    disk = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.5, W / 8.0))
    bulge = wl.draw_galaxies(rng, n, W, 1, r_e_range=(0.3, W / 16.0))
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    out = gfc.gfc_render_stamps(ctx, psf, mix, disk.x, disk.y, disk.flux, disk.r_e, disk.e1, disk.e2, W,
                                mix_id=disk.mix_id)
    gfc.gfc_render_stamps(ctx, psf, mix, bulge.x, bulge.y, bulge.flux, bulge.r_e, bulge.e1, bulge.e2, W,
                          mix_id=bulge.mix_id, flags=gfc.GFC_ACCUMULATE, out=out)
    gpu = _np(out)
    P = cfg["psf"].astype(np.float64)
    idx = list(range(n))
    ref_d = o.render_batch(P, cfg["mix"].as_f32(), disk, idx=idx)
    ref_b = o.render_batch(P, cfg["mix"].as_f32(), bulge, idx=idx)
    _check(gpu, [a + b for a, b in zip(ref_d, ref_b)], idx)
    psf.close(); mix.close()


def test_profile_errors(ctx):
    import paper_2012_15797_amd as gfc
    cfg = wl.config_composite(4)
    gal = cfg["gal"]
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    one = np.ones(4, np.float32)
    with pytest.raises(gfc.GfcError):  # table out of range
        gfc.gfc_render_stamps_composite(ctx, psf, mix, 0, 2, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2,
                                        one, one, 64)
    big = gfc.Mixture(ctx, [10, 8], np.ones((2, 16)) / 10, np.ones((2, 16)))
    with pytest.raises(gfc.GfcError):  # 18 components
        gfc.gfc_render_stamps_composite(ctx, psf, big, 0, 1, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2,
                                        one, one, 64)
    with pytest.raises(gfc.GfcError):  # grid not increasing
        gfc.SersicFamily(ctx, [1.0, 1.0], np.ones((2, 3)), np.ones((2, 3)))
    psf.close(); mix.close(); big.close()


def test_sersic_with_eigen_psf_and_lanczos(ctx):
    """The profile, PSF and shift options compose: general Sersic galaxies
    with a spatially varying PSF and the Lanczos shift, against the oracle
    (eigen PSF at the position, Sersic mixture, Lanczos route)."""
    import paper_2012_15797_amd as gfc
    from oracle import eigen as oe
    from oracle import lanczos as ol
    rng = np.random.Generator(np.random.PCG64(1040))
    fam = wl.sersic_family()
    eig = wl.eigen_psf_moffat(64, 2)
    n = 12
    gal = wl.draw_galaxies(rng, n, 64, 0, r_e_range=(0.5, 6.0))
    sn = rng.uniform(0.5, 6.0, n).astype(np.float32)
    px = rng.uniform(0, 4096, n).astype(np.float32)
    py = rng.uniform(0, 4096, n).astype(np.float32)
    psf = gfc.Psf.eigen(ctx, eig["comps"], eig["coef"], eig["degree"], eig["norm"])
    f = gfc.SersicFamily.from_workload(ctx, fam)
    out = gfc.gfc_render_stamps_sersic(ctx, psf, f, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, sn, 64,
                                       flags=gfc.GFC_SHIFT_LANCZOS3, psf_x=px, psf_y=py)
    gpu = _np(out)
    comps = np.asarray(eig["comps"], np.float32).astype(np.float64)
    ref = []
    for i in range(n):
        p = gal.params(i)
        P = oe.eigen_psf_image(comps, eig["coef"], 2, eig["norm"], float(px[i]), float(py[i]))
        a, v = osr.sersic_mixture(fam["n_grid"], fam["amp"], fam["var"], float(sn[i]))
        ref.append(ol.render_stamp_lanczos(o.psf_spectrum(P, 64), o.psf_gauss_moments(P), a, v, p["x"], p["y"],
                                           p["flux"], p["r_e"], p["e1"], p["e2"], 64))
    _check(gpu, ref, list(range(n)))
    psf.close(); f.close()
