"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with a
library routine, a closed form derived independently, an invariant, or brute
force.  Section references are to Lang (2020), arXiv:2012.15797.
"""

import math

import numpy as np
import pytest

import oracle as o
import workloads as wl


# ---------------------------------------------------------------- steps 1-2
@pytest.mark.parametrize("W", [16, 32, 64, 128])
def test_fold_equals_pad_and_roll_or_periodic_sum(W, rng):
    """Step 1 (embed the PSF): for W >= S the fold is zero padding with the
    centre pixel rolled to index 0; for W < S it is the periodic sum."""
    S = 64
    P = rng.random((S, S))
    Q = o.fold_psf(P, W)
    assert Q.sum() == pytest.approx(P.sum(), rel=1e-14)
    if W >= S:
        pad = np.zeros((W, W))
        pad[:S, :S] = P
        ref = np.roll(pad, (-(S // 2), -(S // 2)), axis=(0, 1))
        np.testing.assert_array_equal(Q, ref)
    else:
        ref = np.zeros((W, W))
        for r in range(S):
            for c in range(S):
                ref[(r - S // 2) % W, (c - S // 2) % W] += P[r, c]
        np.testing.assert_allclose(Q, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("W", [16, 64, 256])
def test_psf_spectrum_matches_library_fft(W, rng):
    """Step 2: the naive DFT equals numpy.fft.fft2 of the embedded PSF."""
    P = rng.random((64, 64))
    ref = np.fft.fft2(o.fold_psf(P, W))
    np.testing.assert_allclose(o.psf_spectrum(P, W), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("W", [16, 64])
def test_inverse_dft_matches_library_ifft(W, rng):
    """Step 7 inverse transform equals numpy.fft.ifft2 (same 1/W^2 scale)."""
    X = rng.standard_normal((W, W)) + 1j * rng.standard_normal((W, W))
    np.testing.assert_allclose(o.inverse_dft2(X), np.fft.ifft2(X), rtol=0, atol=1e-13)


def test_psf_moments_of_sampled_gaussian():
    """Reading R6: moments of a well-sampled offset anisotropic Gaussian are
    its mean and covariance (Poisson summation: exact to ~1e-12)."""
    S = 64
    y, x = np.mgrid[0:S, 0:S].astype(float)
    mx, my, cxx, cxy, cyy = 0.3, -0.2, 3.0, 0.7, 2.0
    det = cxx * cyy - cxy * cxy
    ux, uy = x - S // 2 - mx, y - S // 2 - my
    P = 2.5 * np.exp(-0.5 * (cyy * ux * ux - 2 * cxy * ux * uy + cxx * uy * uy) / det) / (
        2 * math.pi * math.sqrt(det))
    g = o.psf_gauss_moments(P)
    np.testing.assert_allclose(g, [mx, my, cxx, cxy, cyy, 2.5], rtol=1e-9, atol=1e-10)


# ---------------------------------------------------------------- step 3
def _appendix(r_e, e1, e2, t, u, v, w, printed_c12=False):
    """Appendix A: C = v f [[C11, C12], [C12, C22]] for unit mixture variance,
    with c^2, s^2, cs from the trig-free identities of the appendix."""
    e = math.hypot(e1, e2)
    beta = (1 - e) / (1 + e)
    c2, s2, cs = 0.5 * (1 + e1 / e), 0.5 * (1 - e1 / e), e2 / (2 * e)
    f = (r_e / (t * w - u * v)) ** 2
    C11 = beta**2 * (w * w * c2 + 2 * u * w * cs + u * u * s2) + u * u * c2 - 2 * u * w * cs + w * w * s2
    C22 = beta**2 * (v * v * c2 + 2 * t * v * cs + t * t * s2) + t * t * c2 - 2 * t * v * cs + v * v * s2
    if printed_c12:
        # the typeset line: its beta^2 bracket has (u v + t v)
        C12 = -beta**2 * (v * w * c2 + (u * v + t * v) * cs + t * u * s2) - t * u * c2 + (u * v + t * w) * cs - v * w * s2
    else:
        # the commented-out line just above it, which expands A A^T
        C12 = -beta**2 * (v * w * c2 + u * v * cs + t * w * cs + t * u * s2) - v * w * s2 + u * v * cs + t * w * cs - t * u * c2
    return f * np.array([[C11, C12], [C12, C22]])


def test_covariances_match_appendix_a(rng):
    """Eq. C = A V A^T (Section 2 step 3) against Appendix A's written-out
    terms for random CD matrices, ellipticities and radii."""
    for _ in range(50):
        r_e = rng.uniform(0.5, 5)
        e1, e2 = rng.uniform(-0.6, 0.6, 2)
        cd = rng.standard_normal(4)
        v = rng.uniform(0.1, 3)
        a, b, d = o.covariances(r_e, e1, e2, [v], cd)
        ref = v * _appendix(r_e, e1, e2, *cd)
        np.testing.assert_allclose([a[0], b[0], d[0]], [ref[0, 0], ref[0, 1], ref[1, 1]],
                                   rtol=1e-10, atol=1e-12 * abs(ref).max())


def test_appendix_printed_c12_has_a_typo():
    """Reading of the Appendix: the typeset C_12 differs from A A^T (with
    CD = I it drops the -beta^2 c s term); the oracle follows the product."""
    r_e, e1, e2 = 2.0, 0.3, 0.2
    good = _appendix(r_e, e1, e2, 1.0, 0.0, 0.0, 1.0)
    bad = _appendix(r_e, e1, e2, 1.0, 0.0, 0.0, 1.0, printed_c12=True)
    a, b, d = o.covariances(r_e, e1, e2, [1.0])
    assert b[0] == pytest.approx(good[0, 1], rel=1e-12)
    assert abs(bad[0, 1] - good[0, 1]) > 0.1


def test_covariances_trig_free_closed_form_and_eigenvalues(rng):
    """With CD = I, C = v r_e^2/(1+e)^2 [[1+e^2-2e1, 2e2], [2e2, 1+e^2+2e1]]
    (from the Appendix's c^2, s^2, cs identities) and its eigenvalues are
    v r_e^2 {1, beta^2}; e1 > 0 elongates the profile along pixel y."""
    for _ in range(50):
        r_e = rng.uniform(0.2, 10)
        e1, e2 = rng.uniform(-0.69, 0.69, 2)
        v = rng.uniform(1e-4, 10)
        e = math.hypot(e1, e2)
        a, b, d = o.covariances(r_e, e1, e2, [v])
        s = v * r_e**2 / (1 + e) ** 2
        np.testing.assert_allclose([a[0], b[0], d[0]],
                                   [s * (1 + e * e - 2 * e1), s * 2 * e2, s * (1 + e * e + 2 * e1)],
                                   rtol=1e-12)
        beta = (1 - e) / (1 + e)
        ev = np.linalg.eigvalsh(np.array([[a[0], b[0]], [b[0], d[0]]]))
        np.testing.assert_allclose(ev, v * r_e**2 * np.array([beta**2, 1.0]), rtol=1e-10)
    a, b, d = o.covariances(1.0, 0.5, 0.0, [1.0])
    assert d[0] > a[0]
    a0, b0, d0 = o.covariances(3.0, 0.0, 0.0, [2.0])
    assert (a0[0], b0[0], d0[0]) == pytest.approx((18.0, 0.0, 18.0))


# ---------------------------------------------------------------- step 4
def test_routing_ramp_ends_and_smoothness():
    """Step 4: w = 1 at n >= 4, 0 at n <= 3, continuous with zero slope at
    both ends (continuous first derivatives of the profile)."""
    W = 64
    n = np.array([2.0, 3.0, 3.5, 4.0, 5.0])
    tr = ((W / 2) / n) ** 2
    w = o.routing_weights(tr / 2, tr / 2, W)
    np.testing.assert_allclose(w, [0, 0, 0.5, 1, 1], atol=1e-12)
    h = 1e-6
    for n0 in (3.0, 4.0):
        wp = o.routing_weights(*(2 * [((W / 2) / (n0 + h)) ** 2 / 2]), W)
        wm = o.routing_weights(*(2 * [((W / 2) / (n0 - h)) ** 2 / 2]), W)
        assert abs(wp - wm) / (2 * h) < 1e-5
    assert o.routing_weights([100.0], [100.0], W, o.FORCE_FOURIER)[0] == 1.0
    assert o.routing_weights([1e-3], [1e-3], W, o.FORCE_REAL)[0] == 0.0
    lin = o.routing_weights(*(2 * [((W / 2) / 3.25) ** 2 / 2]), W, o.RAMP_LINEAR)
    assert lin == pytest.approx(0.25)


def test_routing_on_workloads():
    """Tiny case: every component is Fourier-side; large-galaxy case: 1-4 of
    8 components touch real space (the paper says typically 1-3)."""
    c = wl.config1()
    amp, var = c["mix"].table(0)
    a, b, d = o.covariances(3.0, 0.2, -0.1, var)
    assert (o.routing_weights(a, d, 64) == 1).all()
    assert ((32 / np.sqrt(a + d)).min()) > 5.0
    c3 = wl.config3(300)
    amp, var = c3["mix"].table(0)
    kr = []
    for i in range(300):
        p = c3["gal"].params(i)
        a, b, d = o.covariances(p["r_e"], p["e1"], p["e2"], var)
        kr.append(int((o.routing_weights(a, d, p["W"]) < 1).sum()))
    kr = np.array(kr)
    assert kr.min() >= 1 and kr.max() <= 4
    assert np.bincount(kr).argmax() == 2
