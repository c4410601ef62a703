"""Pins of the Lanczos sub-pixel-shift oracle (Section 2, step 8: the
optional pixel-space shift used instead of the Fourier phase).

The kernel is pinned by its defining properties: interpolation at the
integers, support, symmetry.  The shift is pinned by exact identities (f = 0,
constants) and by shifting a sampled smooth function, against the sampled
analytically shifted function: a wrong direction, a wrong tap set or a
missing normalisation fails by a wide margin."""

import math

import numpy as np
import pytest

import oracle as o
from oracle import lanczos as ol
import workloads as wl


def test_kernel_interpolates_and_has_support_three():
    assert ol.lanczos3(0.0) == 1.0
    for n in (1, 2, -1, -2):
        assert abs(ol.lanczos3(n)) < 1e-16
    for t in (3.0, -3.0, 3.5, 10.0):
        assert ol.lanczos3(t) == 0.0
    for t in (0.3, 1.7, 2.9):
        assert ol.lanczos3(t) == ol.lanczos3(-t)
    assert abs(ol.lanczos3(2.999999)) < 1e-5  # continuous at the support edge
    # a known value: L(1/2) = sinc(1/2) sinc(1/6) = (2/pi) * (6/pi) sin(pi/6)
    assert abs(ol.lanczos3(0.5) - (2 / math.pi) * (6 / math.pi) * 0.5) < 1e-15


def test_weights_are_normalised_and_reduce_to_identity_at_zero():
    for f in (0.0, 0.1, 0.5, 0.77, 0.999):
        w = ol.lanczos_weights(f)
        assert w.shape == (6,) and abs(w.sum() - 1.0) < 1e-15
    assert np.array_equal(ol.lanczos_weights(0.0), np.array([0, 0, 0, 1, 0, 0], float))


def test_zero_shift_is_identity_and_constants_are_kept_inside():
    rng = np.random.Generator(np.random.PCG64(5))
    img = rng.standard_normal((32, 32))
    assert np.array_equal(ol.lanczos_shift(img, 0.0, 0.0), img)
    out = ol.lanczos_shift(np.full((32, 32), 2.5), 0.37, 0.81)
    assert np.abs(out[3:-3, 3:-3] - 2.5).max() < 1e-14
    # zero outside the stamp (reading L4): at the last column the taps d = 1, 2 fall outside
    wx = ol.lanczos_weights(0.37)
    assert abs(out[10, -1] - 2.5 * wx[:4].sum()) < 1e-14 and abs(wx[4:].sum()) > 1e-3


@pytest.mark.parametrize("fx,fy", [(0.3, 0.7), (0.5, 0.5), (0.9, 0.1), (0.25, 0.0)])
def test_shift_moves_a_smooth_function_by_the_offset(fx, fy):
    """A sampled Gaussian (sigma 2.5 px) shifted by (fx, fy) matches the
    Gaussian sampled at the shifted centre to 0.6% of the peak (Lanczos-3's
    interpolation error at these frequencies is about 0.35%); shifting the
    other way, or by a tap too many, misses by more than 10%."""
    W = 64
    y, x = np.mgrid[0:W, 0:W].astype(float)
    g = lambda cx, cy: np.exp(-0.5 * ((x - cx) ** 2 + (y - cy) ** 2) / 2.5**2)
    out = ol.lanczos_shift(g(31.2, 32.4), fx, fy)
    assert np.abs(out - g(31.2 + fx, 32.4 + fy)).max() <= 6e-3
    assert np.abs(out - g(31.2 - fx, 32.4 - fy)).max() > 0.1 or (fx, fy) == (0.0, 0.0)


def test_integer_position_render_equals_fourier_render():
    P = wl.psf_moffat_halo(64)
    S, gauss = o.psf_spectrum(P, 64), o.psf_gauss_moments(P)
    amp, var = np.array([0.6, 0.4]), np.array([0.05, 3.0])
    args = (amp, var, 31.0, 30.0, 4.0, 2.0, 0.1, 0.2, 64)
    assert np.array_equal(ol.render_stamp_lanczos(S, gauss, *args), o.render_stamp(S, gauss, *args))


def test_tiny_galaxy_is_the_shifted_point_source():
    """Section 2: with Lanczos shifting a galaxy of tiny radius becomes the
    point source, i.e. the PSF rolled to the integer position and shifted by
    the same Lanczos rule."""
    P = wl.psf_moffat_halo(64)
    S, gauss = o.psf_spectrum(P, 64), o.psf_gauss_moments(P)
    x, y, flux = 30.35, 33.8, 2.0
    img = ol.render_stamp_lanczos(S, gauss, np.array([1.0]), np.array([1.0]), x, y, flux, 1e-4, 0.0, 0.0, 64,
                                  o.FORCE_FOURIER)
    point = flux * np.roll(np.roll(o.fold_psf(P, 64), 33, axis=0), 30, axis=1)
    ref = ol.lanczos_shift(point, x - 30, y - 33)
    assert np.abs(img - ref).max() <= 1e-7 * ref.max()
