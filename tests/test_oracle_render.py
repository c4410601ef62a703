"""Whole-stamp pins of the FP64 oracle (Lang 2020, Section 2, steps 5-8).

Each test checks the oracle against a result fixed independently of it: the
closed-form convolution of two Gaussian mixtures, exact invariants of the
DFT (flux, integer shift, transpose), brute-force supersampled quadrature,
and agreement between the Fourier and real-space routes.
"""

import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


def _gauss_mixture_psf(S, sigmas, weights):
    """Unnormalised pixel samples of sum_j w_j N(0, s_j^2 I) about (S/2, S/2)."""
    y, x = np.mgrid[0:S, 0:S].astype(float) - S // 2
    return sum(w * np.exp(-0.5 * (x * x + y * y) / s**2) / (2 * math.pi * s**2)
               for w, s in zip(weights, sigmas))


def _periodized_gaussian(W, x0, y0, cxx, cxy, cyy, images=2):
    y, x = np.mgrid[0:W, 0:W].astype(float)
    det = cxx * cyy - cxy * cxy
    out = np.zeros((W, W))
    for m in range(-images, images + 1):
        for n in range(-images, images + 1):
            ux, uy = x + m * W - x0, y + n * W - y0
            out += np.exp(-0.5 * (cyy * ux * ux - 2 * cxy * ux * uy + cxx * uy * uy) / det)
    return out / (2 * math.pi * math.sqrt(det))


def _render(P, gauss, amp, var, x, y, flux, r_e, e1, e2, W, flags=0):
    return o.render_stamp(o.psf_spectrum(P, W), gauss, amp, var, x, y, flux, r_e, e1, e2, W, flags)


@pytest.mark.parametrize("W,x0,y0,r_e", [(64, 32.3, 31.7, 2.0), (32, 16.0, 16.5, 1.2),
                                         (16, 8.25, 8.75, 0.8)])
def test_closed_form_mog_psf(W, x0, y0, r_e):
    """T1: with a PSF that is pixel samples of a Gaussian mixture, the
    Fourier path equals the periodised analytic sum_ij F A_i w_j
    N(x - mu; C_i + s_j^2 I) at pixel centres ('exact for each Gaussian as
    long as the PSF is well sampled', Section 2).  The residual is the PSF's
    power beyond Nyquist (~1e-6 of the DC term for s = 1.7 px)."""
    sig, wts = (1.7, 4.0), (0.9, 0.1)
    P = _gauss_mixture_psf(64, sig, wts)
    amp = np.array([0.5, 0.3, 0.2])
    var = np.array([0.3, 1.0, 2.5])
    flux, e1, e2 = 3.0, 0.25, -0.15
    img = _render(P, o.psf_gauss_moments(P), amp, var, x0, y0, flux, r_e, e1, e2, W,
                  o.FORCE_FOURIER)
    a, b, d = o.covariances(r_e, e1, e2, var)
    ref = np.zeros((W, W))
    for i in range(3):
        for s, wj in zip(sig, wts):
            ref += flux * amp[i] * wj * _periodized_gaussian(W, x0, y0, a[i] + s * s, b[i], d[i] + s * s)
    err = np.abs(img - ref).max() / ref.max()
    assert err < 5e-8, err


def test_flux_conservation_exact():
    """T2: the DC bin fixes the total: sum(I_F) = F * sum(w_i A_i) * sum(P)."""
    c = wl.config_metric(8)
    amp, var = c["mix"].table(0)
    P = c["psf"].astype(np.float64) * 1.7
    for i in range(8):
        p = c["gal"].params(i)
        img = _render(P, None or o.psf_gauss_moments(P), amp, var, p["x"], p["y"], p["flux"],
                      p["r_e"], p["e1"], p["e2"], 64, o.FORCE_FOURIER)
        assert img.sum() == pytest.approx(p["flux"] * amp.sum() * P.sum(), rel=1e-12)


@pytest.mark.parametrize("dx,dy", [(1, 0), (0, 1), (3, -2), (64, 0)])
def test_integer_shift_is_exact_roll(dx, dy):
    """T3 (shift theorem): moving the centre by whole pixels rolls the
    all-Fourier stamp exactly, including across the periodic edge."""
    c = wl.config1()
    amp, var = c["mix"].table(0)
    P = wl.psf_moffat_halo(64)
    g = o.psf_gauss_moments(P)
    base = _render(P, g, amp, var, 30.37, 33.81, 2.0, 3.0, 0.3, 0.1, 64, o.FORCE_FOURIER)
    moved = _render(P, g, amp, var, 30.37 + dx, 33.81 + dy, 2.0, 3.0, 0.3, 0.1, 64, o.FORCE_FOURIER)
    np.testing.assert_allclose(moved, np.roll(base, (dy, dx), axis=(0, 1)), rtol=0,
                               atol=1e-12 * base.max())


def test_point_source_limit_is_rolled_psf():
    """T4: r_e -> 0 at an integer position gives flux x (embedded PSF)
    centred on that pixel (Section 1's point-source limit)."""
    P = wl.psf_moffat_halo(64)
    amp, var = np.array([0.6, 0.4]), np.array([1.0, 2.0])
    img = _render(P, o.psf_gauss_moments(P), amp, var, 20.0, 41.0, 5.0, 1e-5, 0.2, 0.1, 64,
                  o.FORCE_FOURIER)
    ref = 5.0 * np.roll(o.fold_psf(P, 64), (41, 20), axis=(0, 1))
    np.testing.assert_allclose(img, ref, rtol=0, atol=1e-8 * ref.max())


def test_subpixel_motion_is_pure_phase():
    """T5: sub-pixel motion changes only the phase of each non-Nyquist DFT
    bin, by exp(-2 pi i k dx / W): the rendered galaxy moves smoothly (a
    naive pixel-centre render would jump; Section 1)."""
    c = wl.config1()
    amp, var = c["mix"].table(0)
    P = wl.psf_double_gaussian(64)
    g = o.psf_gauss_moments(P)
    base = np.fft.fft2(_render(P, g, amp, var, 32.0, 32.0, 1.0, 3.0, 0.2, -0.1, 64, o.FORCE_FOURIER))
    k = np.fft.fftfreq(64)
    KX, KY = np.meshgrid(k, k)
    ok = (np.abs(KX) < 0.5) & (np.abs(KY) < 0.5) & (np.abs(base) > 1e-9 * np.abs(base).max())
    for dx, dy in [(0.25, 0.0), (0.5, 0.75), (0.75, 0.25)]:
        F = np.fft.fft2(_render(P, g, amp, var, 32.0 + dx, 32.0 + dy, 1.0, 3.0, 0.2, -0.1, 64,
                                o.FORCE_FOURIER))
        expect = base * np.exp(-2j * math.pi * (KX * dx + KY * dy))
        np.testing.assert_allclose(F[ok], expect[ok], rtol=0, atol=1e-11 * np.abs(base).max())


def test_supersampled_brute_force_tiny_stamp():
    """T6: 16x16 stamp vs brute-force midpoint-rule convolution of the
    continuous galaxy mixture with the continuous PSF on a 16x finer
    periodic grid (the super-resolution route the paper avoids)."""
    W, ss = 16, 16
    sig, wts = (1.7, 4.0), (0.9, 0.1)
    P = _gauss_mixture_psf(64, sig, wts)
    amp, var = np.array([0.7, 0.3]), np.array([0.5, 1.5])
    x0, y0, r_e, e1, e2, flux = 7.3, 8.6, 0.6, 0.3, 0.2, 1.0
    img = _render(P, o.psf_gauss_moments(P), amp, var, x0, y0, flux, r_e, e1, e2, W, o.FORCE_FOURIER)
    a, b, d = o.covariances(r_e, e1, e2, var)
    h = 1.0 / ss
    t = (np.arange(W * ss) + 0.5) * h - 0.5       # fine-grid midpoints over one period
    TX, TY = np.meshgrid(t, t)
    gal = np.zeros_like(TX)
    for i in range(2):
        det = a[i] * d[i] - b[i] ** 2
        for m in (-1, 0, 1):
            for n in (-1, 0, 1):
                ux, uy = TX + m * W - x0, TY + n * W - y0
                gal += amp[i] * np.exp(-0.5 * (d[i] * ux * ux - 2 * b[i] * ux * uy + a[i] * uy * uy) / det) / (
                    2 * math.pi * math.sqrt(det))
    ref = np.zeros((W, W))
    for r in range(W):
        for c in range(W):
            dx = (c - TX + W / 2) % W - W / 2
            dy = (r - TY + W / 2) % W - W / 2
            psf = np.zeros_like(TX)
            for m in (-1, 0, 1):
                for n in (-1, 0, 1):
                    qx, qy = dx + m * W, dy + n * W
                    psf += sum(wj * np.exp(-0.5 * (qx * qx + qy * qy) / s**2) / (2 * math.pi * s**2)
                               for s, wj in zip(sig, wts))
            ref[r, c] = flux * (psf * gal).sum() * h * h
    err = np.abs(img - ref).max() / ref.max()
    assert err < 5e-8, err


def test_transpose_symmetry():
    """T8: transposing the stamp equals swapping x <-> y and e1 -> -e1 when
    the PSF is symmetric under transposition (Nyquist reading R4 keeps this
    exact), on the hybrid path too."""
    P = wl.psf_moffat_halo(64)
    g = o.psf_gauss_moments(P)
    amp, var = wl.dev8_table(np.random.Generator(np.random.PCG64(7)))
    A = _render(P, g, amp, var, 30.3, 33.6, 4.0, 6.0, 0.3, 0.25, 64)
    B = _render(P, g, amp, var, 33.6, 30.3, 4.0, 6.0, -0.3, 0.25, 64)
    np.testing.assert_allclose(A.T, B, rtol=0, atol=1e-12 * A.max())


def test_real_space_route_agrees_with_fourier_route():
    """T10: with a single-Gaussian PSF (so its Gaussian approximation is
    exact) and a component far from the stamp edge, forcing the real-space
    route reproduces the Fourier route (Section 2 step 8)."""
    s = 1.8
    P = _gauss_mixture_psf(64, (s,), (1.0,))
    gauss = np.array([0.0, 0.0, s * s, 0.0, s * s, P.sum()])
    amp, var = np.array([0.6, 0.4]), np.array([0.4, 1.2])
    args = (amp, var, 64.4, 63.7, 10.0, 3.0, 0.2, 0.35, 128)
    F = _render(P, gauss, *args, flags=o.FORCE_FOURIER)
    R = _render(P, gauss, *args, flags=o.FORCE_REAL)
    err = np.abs(F - R).max() / F.max()
    assert err < 1e-7, err


def test_hybrid_beats_small_fft_against_large_fft():
    """T11 (Fig. 2 analogue): a 32x32 hybrid stamp matches the central
    32x32 of a 128x128 all-Fourier render far better than a 32x32
    all-Fourier render, which suffers wrap-around."""
    P = wl.psf_double_gaussian(64)
    g = o.psf_gauss_moments(P)
    amp, var = wl.dev8_table(np.random.Generator(np.random.PCG64(3)))
    big = _render(P, g, amp, var, 64.3, 64.6, 1.0, 6.0, 0.2, 0.1, 128, o.FORCE_FOURIER)
    ref = big[48:80, 48:80]
    fft32 = _render(P, g, amp, var, 16.3, 16.6, 1.0, 6.0, 0.2, 0.1, 32, o.FORCE_FOURIER)
    hyb32 = _render(P, g, amp, var, 16.3, 16.6, 1.0, 6.0, 0.2, 0.1, 32)
    e_fft = np.abs(fft32 - ref).max()
    e_hyb = np.abs(hyb32 - ref).max()
    assert e_hyb < 0.2 * e_fft, (e_hyb, e_fft)


def test_naive_pixel_render_aliases_but_method_does_not():
    """T13 (Fig. 3 analogue): a compact galaxy evaluated at pixel centres and
    FFT-convolved with the PSF has a centroid that lags the true sub-pixel
    position; the method's centroid follows it."""
    P = wl.psf_double_gaussian(64)
    g = o.psf_gauss_moments(P)
    amp, var = np.array([0.5, 0.5]), np.array([0.01, 0.05])
    W = 64
    yy, xx = np.mgrid[0:W, 0:W].astype(float)
    Q = o.fold_psf(P, W)
    errs_m, errs_n = [], []
    for dx in (0.0, 0.2, 0.4, 0.6, 0.8):
        x0 = 32.0 + dx
        img = _render(P, g, amp, var, x0, 32.0, 1.0, 1.0, 0.0, 0.0, W, o.FORCE_FOURIER)
        naive_gal = sum(ai * np.exp(-0.5 * ((xx - x0) ** 2 + (yy - 32.0) ** 2) / vi) / (2 * math.pi * vi)
                        for ai, vi in zip(amp, var))
        naive = np.real(np.fft.ifft2(np.fft.fft2(naive_gal) * np.fft.fft2(Q)))
        cm = (img * xx).sum() / img.sum()
        cn = (naive * xx).sum() / naive.sum()
        errs_m.append(abs(cm - x0))
        errs_n.append(abs(cn - x0))
    assert max(errs_m) < 1e-6
    assert max(errs_n) > 1e-2


def test_invalid_parameters_give_nan_stamp():
    """Reading R8: |e| >= 1, r_e <= 0 or non-finite values -> NaN stamp."""
    P = wl.psf_double_gaussian(64)
    ph = o.psf_spectrum(P, 16)
    g = o.psf_gauss_moments(P)
    for bad in [dict(e1=0.8, e2=0.7), dict(r_e=0.0), dict(x=float("nan"))]:
        p = dict(x=8.0, y=8.0, flux=1.0, r_e=1.0, e1=0.1, e2=0.1)
        p.update(bad)
        img = o.render_stamp(ph, g, [1.0], [1.0], W=16, **p)
        assert np.isnan(img).all()


def test_real_space_route_off_centre_elliptical_psf():
    """T10 with an off-centre, elliptical single-Gaussian PSF (mean
    (0.37, -0.21) px from the centre pixel, covariance with a cross term).
    The Fourier route sees the PSF only through its pixels (steps 1-2), the
    real-space route only through the explicit description (step 8), so
    their agreement pins the description's mean and cross term in step 8:
    a sign error in either moves the real-space image by over 10% of the
    peak.  Both also match the periodised analytic Gaussian centred at
    x0 + mu_p with covariance C_i + Sigma_p."""
    P, gauss = wl.psf_offset_gaussian(64)
    amp, var = np.array([0.6, 0.4]), np.array([0.4, 1.2])
    x0, y0, flux, r_e, e1, e2, W = 64.4, 63.7, 10.0, 3.0, 0.2, 0.35, 128
    args = (amp, var, x0, y0, flux, r_e, e1, e2, W)
    F = _render(P, gauss, *args, flags=o.FORCE_FOURIER)
    R = _render(P, gauss, *args, flags=o.FORCE_REAL)
    assert np.abs(F - R).max() / F.max() < 1e-8
    a, b, d = o.covariances(r_e, e1, e2, var)
    mux, muy, pxx, pxy, pyy, _ = gauss
    ref = sum(flux * amp[i] * _periodized_gaussian(W, x0 + mux, y0 + muy, a[i] + pxx, b[i] + pxy,
                                                   d[i] + pyy, images=1) for i in range(2))
    assert np.abs(F - ref).max() / F.max() < 1e-8
    # the hybrid route splits ramped components between the two; with a stamp
    # small enough to ramp them the sum still matches the all-Fourier render of
    # the same galaxy in a stamp large enough not to wrap
    big = _render(P, gauss, amp, var, 64.4, 63.7, flux, 6.0, e1, e2, 128, o.FORCE_FOURIER)
    hyb = _render(P, gauss, amp, var, 16.4, 15.7, flux, 6.0, e1, e2, 32)
    parts = o.render_stamp(o.psf_spectrum(P, 32), gauss, amp, var, 16.4, 15.7, flux, 6.0, e1, e2, 32,
                           return_parts=True)[1]
    w = parts["w"]
    assert np.any((w > 0) & (w < 1)) and np.any(w == 0), w        # one ramped, one real-space
    fft32 = _render(P, gauss, amp, var, 16.4, 15.7, flux, 6.0, e1, e2, 32, o.FORCE_FOURIER)
    e_hyb = np.abs(hyb - big[48:80, 48:80]).max() / big.max()
    e_fft = np.abs(fft32 - big[48:80, 48:80]).max() / big.max()
    assert e_hyb < 2e-4 and e_hyb < 0.02 * e_fft, (e_hyb, e_fft)
