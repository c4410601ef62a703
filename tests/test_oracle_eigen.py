"""Pins of the eigen-PSF oracle (spatially varying PSF; Section 2, the
step-2 discussion of component PSF models with polynomial amplitudes).

The varying PSF is checked through closed forms: with components that are
pixel samples of Gaussians, the stamp at any position is the analytic
convolution of the galaxy mixture with the position's Gaussian mixture PSF,
so each polynomial term's weight is visible in the result."""

import math

import numpy as np
import pytest

import oracle as o
from oracle import eigen as oe
import workloads as wl


def _gauss(S, s):
    y, x = np.mgrid[0:S, 0:S].astype(float) - S // 2
    return np.exp(-0.5 * (x * x + y * y) / s**2) / (2 * math.pi * s**2)


def _periodized_gaussian(W, x0, y0, cxx, cxy, cyy, images=2):
    y, x = np.mgrid[0:W, 0:W].astype(float)
    det = cxx * cyy - cxy * cxy
    out = np.zeros((W, W))
    for m in range(-images, images + 1):
        for n in range(-images, images + 1):
            ux, uy = x + m * W - x0, y + n * W - y0
            out += np.exp(-0.5 * (cyy * ux * ux - 2 * cxy * ux * uy + cxx * uy * uy) / det)
    return out / (2 * math.pi * math.sqrt(det))


SIG = (1.7, 2.2, 1.4)


def _comps(S=64):
    g = [_gauss(S, s) for s in SIG]
    # a base PSF and two width perturbations, as an eigen decomposition would give
    return np.stack([g[0], g[1] - g[0], g[2] - g[0]])


def test_single_constant_component_is_the_plain_render():
    """J = 1, degree 0, weight 1: the eigen render is the constant-PSF render."""
    P = wl.psf_moffat_halo(64)
    amp, var = np.array([0.6, 0.4]), np.array([0.5, 2.0])
    args = (amp, var, 30.4, 33.1, 5.0, 2.5, 0.2, -0.1, 64)
    ref = o.render_stamp(o.psf_spectrum(P, 64), o.psf_gauss_moments(P), *args)
    got = oe.render_stamp_eigen(P[None], [[1.0]], 0, (0.0, 1.0, 0.0, 1.0), 123.0, -45.0, *args)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("t", range(6))
def test_each_polynomial_term_weights_its_component(t):
    """Degree 2 (terms 1, u, u^2, v, uv, v^2): component 1 carries term t and
    component 2 the constant term scaled by 0.3.  The Fourier render must
    equal the analytic periodised mixture with PSF weights
    (1 - c1 - c2, c1, c2) on the Gaussians of widths SIG."""
    W, x0, y0, r_e = 64, 31.3, 32.6, 2.0
    exps = oe.poly_exponents(2)
    assert exps == [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2)]
    coef = np.zeros((3, 6))
    coef[0, 0] = 1.0
    coef[1, t] = 1.0
    coef[2, 0] = 0.3
    norm = (1000.0, 800.0, 2000.0, 1500.0)
    X, Y = 1420.0, 980.0
    u, v = (X - norm[0]) / norm[1], (Y - norm[2]) / norm[3]
    a_, b_ = exps[t]
    c1, c2 = u**a_ * v**b_, 0.3
    amp, var = np.array([0.7, 0.3]), np.array([0.4, 1.5])
    flux, e1, e2 = 2.0, 0.3, 0.1
    img = oe.render_stamp_eigen(_comps(), coef, 2, norm, X, Y, amp, var, x0, y0, flux, r_e, e1, e2, W,
                                o.FORCE_FOURIER)
    a, b, d = o.covariances(r_e, e1, e2, var)
    ref = np.zeros((W, W))
    for i in range(2):
        for wj, s in zip((1.0 - c1 - c2, c1, c2), SIG):
            ref += flux * amp[i] * wj * _periodized_gaussian(W, x0, y0, a[i] + s * s, b[i], d[i] + s * s)
    assert np.abs(img - ref).max() <= 5e-7 * np.abs(ref).max()


def test_position_moves_the_real_space_psf_gaussian():
    """Real-space route (FORCE_REAL) with Gaussian components: the PSF
    Gaussian is the moment Gaussian of the PSF at the position (reading
    E4).  With a width perturbation weighted by u, the moment variance is
    the weighted variance of the mixture, so the stamp equals the analytic
    Gaussian of that single covariance."""
    W, x0, y0 = 64, 32.0, 32.0
    comps = _comps()
    coef = np.zeros((3, 3))
    coef[0, 0] = 1.0
    coef[1, 1] = 1.0  # u
    norm = (0.0, 100.0, 0.0, 100.0)
    X, Y = 40.0, 0.0  # u = 0.4
    P = oe.eigen_psf_image(comps, coef, 1, norm, X, Y)
    mom = o.psf_gauss_moments(P)
    c1 = 0.4
    # moment variance of (1 - c1) N(1.7^2) + c1 N(2.2^2) sampled on the grid
    y, x = np.mgrid[0:64, 0:64].astype(float) - 32
    Pd = (1 - c1) * _gauss(64, 1.7) + c1 * _gauss(64, 2.2)
    assert np.allclose(P, Pd, rtol=0, atol=1e-15)
    vxx = (Pd * x * x).sum() / Pd.sum()
    assert abs(mom[2] - vxx) < 1e-12 and abs(mom[3]) < 1e-12
    amp, var = np.array([1.0]), np.array([0.8])
    img = oe.render_stamp_eigen(comps, coef, 1, norm, X, Y, amp, var, x0, y0, 3.0, 1.5, 0.0, 0.0, W,
                                o.FORCE_REAL)
    a, b, d = o.covariances(1.5, 0.0, 0.0, var)
    ref = 3.0 * Pd.sum() * _periodized_gaussian(W, x0, y0, a[0] + vxx, 0.0, d[0] + vxx, images=0)
    assert np.abs(img - ref).max() <= 1e-12 * ref.max()


def test_fitted_eigen_psf_reproduces_its_samples():
    """The synthetic eigen-PSF generator: the PSF it gives at the fitting
    grid's centre is close to a unit-sum image, and it varies over the field."""
    eig = wl.eigen_psf_moffat(64, 2)
    P0 = oe.eigen_psf_image(eig["comps"], eig["coef"], 2, eig["norm"], 2048.0, 2048.0)
    P1 = oe.eigen_psf_image(eig["comps"], eig["coef"], 2, eig["norm"], 4000.0, 100.0)
    assert abs(P0.sum() - 1.0) < 1e-4 and abs(P1.sum() - 1.0) < 1e-4
    assert np.abs(P0 - P1).max() > 1e-3 * P0.max()
