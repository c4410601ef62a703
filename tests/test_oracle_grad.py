"""Pins of the FP64 derivative oracle: analytic forward-mode derivatives of
the render (oracle/grad.py) against central finite differences of the forward
oracle, on the Fourier, real-space and ramped routes."""

import math

import numpy as np
import pytest

import oracle as o
import workloads as wl
from oracle.grad import PARAMS


def _case(W, flags, r_e, e1, e2, x, y, flux, seed=0):
    P = wl.psf_moffat_halo(64)
    gauss = o.psf_gauss_moments(P)
    amp, var = wl.dev8_table(np.random.Generator(np.random.PCG64(seed)))
    ph = o.psf_spectrum(P, W)
    params = dict(x=x, y=y, flux=flux, r_e=r_e, e1=e1, e2=e2)
    g = np.random.Generator(np.random.PCG64(seed + 1)).standard_normal((W, W))
    return ph, gauss, amp, var, params, g


@pytest.mark.parametrize("W,flags,r_e", [
    (32, o.FORCE_FOURIER, 2.0),   # Fourier route only
    (32, o.FORCE_REAL, 2.0),      # real-space route only
    (32, 0, 3.0),                 # hybrid with ramped components
    (64, 0, 6.0),
    (32, o.RAMP_LINEAR, 3.0),
])
def test_analytic_gradient_matches_central_fd(W, flags, r_e):
    ph, gauss, amp, var, p, g = _case(W, flags, r_e, 0.23, -0.17, W / 2 + 0.31, W / 2 + 0.77, 7.0)
    I, J = o.render_stamp_jacobian(ph, gauss, amp, var, W=W, flags=flags, **p)
    np.testing.assert_allclose(I, o.render_stamp(ph, gauss, amp, var, W=W, flags=flags, **p),
                               rtol=0, atol=1e-13 * np.abs(I).max())
    an = o.loss_gradient(g, J)
    fd = o.fd_gradient(ph, gauss, amp, var, p, W, g, flags=flags, h=1e-4)
    scale = max(abs(an[k]) for k in PARAMS)
    for k in PARAMS:
        assert an[k] == pytest.approx(fd[k], rel=1e-6, abs=1e-8 * scale), k
    np.testing.assert_allclose(an["amp"], fd["amp"], rtol=1e-6, atol=1e-8 * np.abs(an["amp"]).max())


def test_ramp_derivative_is_continuous():
    """Smoothstep routing keeps d(loss)/d(log r_e) continuous as a component
    crosses n = 3 and n = 4 (Section 2 step 4: continuous first derivatives);
    the linear ramp, by contrast, has a jump there."""
    W = 32
    P = wl.psf_moffat_halo(64)
    gauss = o.psf_gauss_moments(P)
    ph = o.psf_spectrum(P, W)
    amp, var = np.array([1.0]), np.array([1.0])
    g = np.random.Generator(np.random.PCG64(5)).standard_normal((W, W))

    def deriv(r, flags):
        _, J = o.render_stamp_jacobian(ph, gauss, amp, var, W / 2 + 0.3, W / 2 - 0.2, 1.0,
                                       r, 0.0, 0.0, W, flags)
        return float(np.sum(g * J["log_re"]))

    for n_edge in (3.0, 4.0):
        r_edge = (W / 2) / n_edge / math.sqrt(2.0)     # e = 0: a + d = 2 v r_e^2
        lo, hi = (deriv(r_edge * math.exp(s), 0) for s in (-1e-9, 1e-9))
        assert abs(lo - hi) < 1e-6 * abs(lo), (n_edge, lo, hi)
        lo, hi = (deriv(r_edge * math.exp(s), o.RAMP_LINEAR) for s in (-1e-9, 1e-9))
        assert abs(lo - hi) > 1e-3 * abs(lo), (n_edge, lo, hi)


@pytest.mark.parametrize("W,flags,r_e", [(32, o.FORCE_REAL, 2.0), (32, 0, 3.0), (64, 0, 6.0)])
def test_analytic_gradient_off_centre_elliptical_psf(W, flags, r_e):
    """The real-space derivatives with a PSF Gaussian whose mean is off the
    centre pixel and whose covariance has a cross term (step 8): the
    Jacobian's image must equal the forward oracle's (pinned against the
    Fourier route for this PSF) and its derivatives the central differences
    of it, so a sign error in the mean or cross term fails here."""
    P, gauss = wl.psf_offset_gaussian(64)
    amp, var = wl.dev8_table(np.random.Generator(np.random.PCG64(11)))
    ph = o.psf_spectrum(P, W)
    p = dict(x=W / 2 + 0.31, y=W / 2 + 0.77, flux=7.0, r_e=r_e, e1=0.23, e2=-0.17)
    g = np.random.Generator(np.random.PCG64(12)).standard_normal((W, W))
    I, J = o.render_stamp_jacobian(ph, gauss, amp, var, W=W, flags=flags, **p)
    np.testing.assert_allclose(I, o.render_stamp(ph, gauss, amp, var, W=W, flags=flags, **p),
                               rtol=0, atol=1e-13 * np.abs(I).max())
    an = o.loss_gradient(g, J)
    fd = o.fd_gradient(ph, gauss, amp, var, p, W, g, flags=flags, h=1e-4)
    scale = max(abs(an[k]) for k in PARAMS)
    for k in PARAMS:
        assert an[k] == pytest.approx(fd[k], rel=1e-6, abs=1e-8 * scale), k
    np.testing.assert_allclose(an["amp"], fd["amp"], rtol=1e-6, atol=1e-8 * np.abs(an["amp"]).max())
