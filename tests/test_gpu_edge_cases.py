"""GPU parity (through the C ABI) on the cases the workloads leave out:

- a PSF whose single-Gaussian description is off the centre pixel and has a
  cross term (step 8's mean and covariance enter the real-space components
  and their derivatives with a sign the centred isotropic PSFs cannot show);
- mixture components with amplitude exactly zero (dL/dA_k does not depend on
  A_k, so the adjoint must still form that component's sums);
- galaxies with e = 0 exactly (the (e1, e2) derivative is taken as 0 there);
- a table with the largest component count, K = 16.

Forward bar: per stamp, max |gpu - oracle| <= 1e-5 x max |oracle|.  Adjoint
bar: that of tests/gpu_helpers.py."""

import numpy as np
import pytest

import oracle as o
import workloads as wl
from gpu_helpers import TOL_PEAK, assert_grads_close, gpu_grads, oracle_grads, peak_errors, render_gpu

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 64, 128, 256]


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


def _offset_psf(ctx, cfg):
    import paper_2012_15797_amd as gfc

    P, gauss = wl.psf_offset_gaussian(64)
    P32 = P.astype(np.float32)
    psf = gfc.Psf(ctx, P32, gauss)
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    return psf, mix, dict(cfg, psf=P32, psf_gauss=gauss)


def _oracle(cfg, gal, flags=0, mix=None):
    P = np.asarray(cfg["psf"], np.float32).astype(np.float64)
    m = cfg["mix"].as_f32() if mix is None else mix
    return o.render_batch(P, m, gal, flags=flags, psf_gauss=cfg.get("psf_gauss"))


@pytest.mark.parametrize("flags", [0, 2], ids=["hybrid", "forced_real"])
@pytest.mark.parametrize("W", SIZES)
def test_off_centre_elliptical_psf_forward(ctx, W, flags):
    """Real-space components with a PSF Gaussian at mu = (0.37, -0.21) px and
    covariance [[3.1, 0.8], [0.8, 2.2]]; radii spread so that the hybrid
    route has Fourier, ramped and real-space components."""
    rng = np.random.Generator(np.random.PCG64(800 + W + flags))
    psf, mix, cfg = _offset_psf(ctx, wl.config2(10))
    n = 40 if W < 256 else 12
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.3, W / 4.0))
    gpu = render_gpu(ctx, psf, mix, gal, W, flags=flags)
    idx = list(range(n))
    errs = peak_errors(gpu, _oracle(cfg, gal, flags), idx)
    assert errs.max() <= TOL_PEAK, (errs.max(), int(errs.argmax()))
    psf.close(); mix.close()


@pytest.mark.parametrize("flags", [0, 2], ids=["hybrid", "forced_real"])
@pytest.mark.parametrize("W", SIZES)
def test_off_centre_elliptical_psf_backward(ctx, W, flags):
    rng = np.random.Generator(np.random.PCG64(850 + W + flags))
    psf, mix, cfg = _offset_psf(ctx, wl.config2(10))
    n = 24 if W < 128 else 6
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g, flags=flags)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, flags=flags)
    assert_grads_close(gp, rp, f"params W={W} flags={flags} offset PSF")
    assert_grads_close(ga, ra, f"amplitudes W={W} flags={flags} offset PSF", scale=ra_abs)
    psf.close(); mix.close()


def _zero_amp_mixture():
    """EXP6 and DEV8 tables with some amplitudes exactly zero: the first, a
    middle and the last component of EXP6, two of DEV8."""
    m = wl.config2(10)["mix"].as_f32()
    amp = np.array(m.amp, np.float32)
    amp[0, [0, 2, int(m.K[0]) - 1]] = 0.0
    amp[1, [1, 5]] = 0.0
    return wl.Mixtures(np.array(m.K), amp.astype(np.float64), np.array(m.var))


@pytest.mark.parametrize("flags", [1, 2, 0], ids=["fourier", "real", "hybrid"])
@pytest.mark.parametrize("W", [32, 64, 256])
def test_zero_amplitude_components_backward(ctx, W, flags):
    """dL/dA_k of a component with A_k = 0 is w_k p_k + (1 - w_k) r_k, not
    zero, on the Fourier, the real-space and the hybrid route."""
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(900 + W + flags))
    cfg = wl.config2(10)
    m = _zero_amp_mixture()
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, m)
    n = 20 if W < 256 else 6
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g, flags=flags)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, flags=flags, mix=m)
    zero = (np.array(m.amp) == 0) & (np.arange(16)[None, :] < np.array(m.K)[:, None])
    assert np.all(np.abs(ra[zero]) > 0)      # the oracle's gradients there are not zero
    assert_grads_close(gp, rp, f"params W={W} flags={flags} zero amplitudes")
    assert_grads_close(ga, ra, f"amplitudes W={W} flags={flags} zero amplitudes", scale=ra_abs)
    psf.close(); mix.close()


@pytest.mark.parametrize("W", SIZES)
def test_round_galaxies_e_zero(ctx, W):
    """e1 = e2 = 0 exactly: forward parity, and the adjoint gives (e1, e2)
    derivatives of 0 (reading: the profile has a cone at e = 0) with every
    other derivative matching the oracle."""
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(950 + W))
    cfg = wl.config2(10)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    n = 16 if W < 256 else 6
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    gal.e1[:] = 0.0
    gal.e2[:] = 0.0
    gpu = render_gpu(ctx, psf, mix, gal, W)
    errs = peak_errors(gpu, _oracle(cfg, gal), list(range(n)))
    assert errs.max() <= TOL_PEAK, errs.max()
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g)
    assert np.all(rp[:, 4:] == 0) and np.all(gp[:, 4:] == 0)
    assert_grads_close(gp[:, :4], rp[:, :4], f"params W={W} e = 0")
    assert_grads_close(ga, ra, f"amplitudes W={W} e = 0", scale=ra_abs)
    psf.close(); mix.close()


def _k16_mixture():
    rng = np.random.Generator(np.random.PCG64(16))
    amp = np.zeros((1, 16), np.float32)
    amp[0] = rng.dirichlet(np.ones(16)).astype(np.float32)
    var = np.zeros((1, 16), np.float32)
    var[0] = np.logspace(-4, 1, 16).astype(np.float32)
    return wl.Mixtures(np.array([16], np.int32), amp.astype(np.float64), var.astype(np.float64))


@pytest.mark.parametrize("W", SIZES)
def test_sixteen_component_table(ctx, W):
    """A table with K = 16 (the largest), forward and adjoint, hybrid route."""
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(1000 + W))
    cfg = wl.config2(10)
    m = _k16_mixture()
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, m)
    n = 24 if W < 256 else 6
    gal = wl.draw_galaxies(rng, n, W, np.zeros(n, np.int32), r_e_range=(0.4, W / 5.0))
    gpu = render_gpu(ctx, psf, mix, gal, W)
    errs = peak_errors(gpu, _oracle(cfg, gal, mix=m), list(range(n)))
    assert errs.max() <= TOL_PEAK, errs.max()
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, mix=m)
    assert_grads_close(gp, rp, f"params W={W} K=16")
    assert_grads_close(ga, ra, f"amplitudes W={W} K=16", scale=ra_abs)
    psf.close(); mix.close()
