"""FP64 oracle of the forward render (Lang 2020, Section 2, steps 1-8).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.

Each function follows one step of the paper's eight-step list and is written
from its definition, with naive DFT matrices (no FFT) and direct evaluation of
every Gaussian.  Where the paper is silent the readings below are used; the
HIP path implements the same readings independently.

Readings (where the paper is silent or ambiguous):
  R1  PSF centre is pixel (S_y/2, S_x/2); it is moved to index 0 and the grid
      is folded periodically modulo W (zero-padding when W >= S).
  R2  Aliasing measure n_i = (W/2) / sqrt(a_i + d_i) (Section 2, step 4 text
      describes sigma over the half-size; its inverse is the sigma count).
  R3  Ramp between n = 3 and 4 is the smoothstep 3t^2 - 2t^3, t = n - 3
      (continuous first derivatives); RAMP_LINEAR selects w = t.
  R4  At the Nyquist index k = W/2 of each axis the galaxy transform is the
      mean of its values at +1/2 and -1/2 (four-way at the corner).
  R5  Real-space components are point-sampled at pixel centres, not wrapped.
  R6  The single-Gaussian PSF approximation is an explicit input
      {mu_x, mu_y, c_xx, c_xy, c_yy, amp}; default is the moments of the
      pixel PSF about its centre pixel, amp = sum of the pixels.
  R7  Pixel (row r, column c) has its centre at (x=c, y=r).
  R8  e = 0 gives C = v r_e^2 I; |e| >= 1, r_e <= 0 or a non-finite
      parameter gives an all-NaN stamp.
"""

from __future__ import annotations

import math

import numpy as np

FORCE_FOURIER = 1
FORCE_REAL = 2
RAMP_LINEAR = 4

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# Steps 1-2: embed the pixelized PSF in the output grid and transform it.
# --------------------------------------------------------------------------

def fold_psf(P: np.ndarray, W: int) -> np.ndarray:
    """Step 1 (embed the PSF in a W x W grid), reading R1.

    Q[(r - S_y/2) mod W, (c - S_x/2) mod W] += P[r, c]: the PSF centre pixel
    lands on index (0, 0); for W >= S this is zero padding, for W < S the
    PSF wraps periodically so its total is kept.  Pinned by: sum conservation
    and a direct comparison with zero-padding + roll (tests)."""
    P = np.asarray(P, np.float64)
    Sy, Sx = P.shape
    Q = np.zeros((W, W), np.float64)
    rows = (np.arange(Sy) - Sy // 2) % W
    cols = (np.arange(Sx) - Sx // 2) % W
    np.add.at(Q, (rows[:, None], cols[None, :]), P)
    return Q


def dft_matrix(W: int, sign: int) -> np.ndarray:
    """F[k, n] = exp(sign * 2 pi i k n / W), with k n reduced mod W exactly."""
    kn = np.outer(np.arange(W), np.arange(W)) % W
    return np.exp(sign * 1j * TWO_PI * kn / W)


def psf_spectrum(P: np.ndarray, W: int) -> np.ndarray:
    """Step 2: DFT of the embedded PSF on the W x W frequency grid.

    P_hat[k_y, k_x] = sum_{r,c} Q[r, c] exp(-2 pi i (k_x c + k_y r) / W),
    computed as two naive DFT-matrix products.  Pinned against
    numpy.fft.fft2 (tests)."""
    Q = fold_psf(P, W)
    F = dft_matrix(W, -1)
    return F @ Q @ F


def psf_gauss_moments(P: np.ndarray) -> np.ndarray:
    """Reading R6: single-Gaussian PSF approximation by moments about the
    centre pixel.  Returns {mu_x, mu_y, c_xx, c_xy, c_yy, amp}.  Pinned by a
    sampled Gaussian whose moments are known (tests)."""
    P = np.asarray(P, np.float64)
    Sy, Sx = P.shape
    y = np.arange(Sy, dtype=np.float64)[:, None] - Sy // 2
    x = np.arange(Sx, dtype=np.float64)[None, :] - Sx // 2
    amp = P.sum()
    mx = (P * x).sum() / amp
    my = (P * y).sum() / amp
    cxx = (P * (x - mx) ** 2).sum() / amp
    cyy = (P * (y - my) ** 2).sum() / amp
    cxy = (P * (x - mx) * (y - my)).sum() / amp
    return np.array([mx, my, cxx, cxy, cyy, amp])


# --------------------------------------------------------------------------
# Step 3: galaxy shape -> pixel-space covariances.
# --------------------------------------------------------------------------

def shape_matrix(r_e: float, e1: float, e2: float, cd=None) -> np.ndarray:
    """Section 2, step 3: theta = atan2(e2, e1)/2, e = |(e1, e2)|,
    beta = (1-e)/(1+e), E = r_e [[beta cos, sin], [-beta sin, cos]] and the
    combined affine matrix A = CD^{-1} E (CD = identity when None)."""
    e = math.hypot(e1, e2)
    theta = 0.5 * math.atan2(e2, e1) if e > 0 else 0.0
    beta = (1.0 - e) / (1.0 + e)
    c, s = math.cos(theta), math.sin(theta)
    E = r_e * np.array([[beta * c, s], [-beta * s, c]])
    if cd is None:
        return E
    return np.linalg.solve(np.asarray(cd, np.float64).reshape(2, 2), E)


def covariances(r_e, e1, e2, var, cd=None):
    """Equation for C (Section 2, step 3): C_i = A (v_i I) A^T for each
    isotropic mixture variance v_i.  Returns (a, b, d) arrays with
    C_i = [[a_i, b_i], [b_i, d_i]], x first.  Pinned against the closed
    forms of Appendix A and the eigenvalues v r_e^2 {1, beta^2} (tests)."""
    A = shape_matrix(r_e, e1, e2, cd)
    B = A @ A.T
    var = np.asarray(var, np.float64)
    return var * B[0, 0], var * B[0, 1], var * B[1, 1]


# --------------------------------------------------------------------------
# Step 4: which components alias.
# --------------------------------------------------------------------------

def routing_weights(a, d, W: int, flags: int = 0) -> np.ndarray:
    """Section 2, step 4, readings R2 and R3: w_i = 1 (Fourier) when
    n_i >= 4, 0 (real space) when n_i <= 3, smoothstep in between.
    Pinned by the ramp's end values and C1 continuity (tests)."""
    a = np.asarray(a, np.float64)
    d = np.asarray(d, np.float64)
    if flags & FORCE_FOURIER:
        return np.ones_like(a)
    if flags & FORCE_REAL:
        return np.zeros_like(a)
    n = (W / 2.0) / np.sqrt(a + d)
    t = np.clip(n - 3.0, 0.0, 1.0)
    if flags & RAMP_LINEAR:
        return t
    return t * t * (3.0 - 2.0 * t)


# --------------------------------------------------------------------------
# Steps 5-6: analytic transform of the shifted mixture on the FFT grid.
# --------------------------------------------------------------------------

def axis_frequencies(W: int):
    """Frequencies of DFT index k on one axis: k/W below W/2, (k-W)/W above.
    Returns two arrays that differ only at the Nyquist index, where one holds
    -1/2 and the other +1/2 (reading R4)."""
    k = np.arange(W, dtype=np.float64)
    f = np.where(k < W / 2, k / W, (k - W) / W)
    lo = f.copy()
    hi = f.copy()
    if W % 2 == 0:
        lo[W // 2] = -0.5
        hi[W // 2] = +0.5
    return lo, hi


def _mixture_ft(nu, om, x0, y0, coef, a, b, d):
    """Eq. for M(nu, omega): phase exp(-2 pi i (x0 nu + y0 omega)) times
    sum_i coef_i exp(-2 pi^2 (a_i nu^2 + 2 b_i nu omega + d_i omega^2))."""
    phase = np.exp(-1j * TWO_PI * (x0 * nu + y0 * om))
    s = np.zeros(nu.shape, np.float64)
    for ci, ai, bi, di in zip(coef, a, b, d):
        if ci == 0.0:
            continue
        s += ci * np.exp(-2.0 * math.pi**2 * (ai * nu * nu + 2.0 * bi * nu * om + di * om * om))
    return phase * s


def galaxy_spectrum(x0, y0, coef, a, b, d, W: int) -> np.ndarray:
    """Steps 5-6: M[k_y, k_x] for every bin of the W x W grid (k_x along the
    columns / x axis, k_y along the rows / y axis), with the Nyquist mean of
    reading R4.  Pinned by the closed-form MoG x MoG-PSF render, flux
    conservation, integer-shift and transpose symmetries (tests)."""
    lo, hi = axis_frequencies(W)
    M = np.zeros((W, W), np.complex128)
    for fx in (lo, hi):
        for fy in (lo, hi):
            NU, OM = np.meshgrid(fx, fy)
            M += _mixture_ft(NU, OM, x0, y0, coef, a, b, d)
    return M / 4.0


def inverse_dft2(X: np.ndarray) -> np.ndarray:
    """Step 7 (inverse): I[r, c] = W^-2 sum_k X[k_y, k_x]
    exp(+2 pi i (k_x c + k_y r) / W), as naive DFT-matrix products.
    Pinned against numpy.fft.ifft2 (tests)."""
    W = X.shape[0]
    F = dft_matrix(W, +1)
    return (F @ X @ F) / (W * W)


# --------------------------------------------------------------------------
# Step 8: components evaluated in real space.
# --------------------------------------------------------------------------

def real_space_image(x0, y0, coef, a, b, d, gauss, W: int) -> np.ndarray:
    """Step 8, readings R5 and R6: sum over components with coef_i != 0 of
    coef_i * amp_p * N((c, r) - (x0, y0) - mu_p; C_i + Sigma_p), with
    N(u; S) = exp(-u^T S^-1 u / 2) / (2 pi sqrt(det S)), point-sampled at
    pixel centres.  Pinned by the closed-form Gaussian convolution and by
    agreement with the Fourier path for large stamps, including a PSF whose
    Gaussian is off the centre pixel and has a cross term, so the signs of
    mu_p and of the covariance's cross term are fixed (tests)."""
    mux, muy, pxx, pxy, pyy, pamp = [float(v) for v in gauss]
    yy, xx = np.mgrid[0:W, 0:W].astype(np.float64)
    ux = xx - x0 - mux
    uy = yy - y0 - muy
    img = np.zeros((W, W), np.float64)
    for ci, ai, bi, di in zip(coef, a, b, d):
        if ci == 0.0:
            continue
        sxx, sxy, syy = ai + pxx, bi + pxy, di + pyy
        det = sxx * syy - sxy * sxy
        q = (syy * ux * ux - 2.0 * sxy * ux * uy + sxx * uy * uy) / det
        img += ci * pamp * np.exp(-0.5 * q) / (TWO_PI * math.sqrt(det))
    return img


# --------------------------------------------------------------------------
# Whole stamp.
# --------------------------------------------------------------------------

def _valid(x, y, flux, r_e, e1, e2) -> bool:
    vals = (x, y, flux, r_e, e1, e2)
    if not all(math.isfinite(v) for v in vals):
        return False
    return r_e > 0.0 and math.hypot(e1, e2) < 1.0


def render_stamp(psf_hat, gauss, amp, var, x, y, flux, r_e, e1, e2, W,
                 flags: int = 0, cd=None, return_parts: bool = False):
    """Steps 3-8 for one galaxy.  psf_hat is psf_spectrum(P, W).

    I = Re(W^-2 IDFT(flux * P_hat * M)) + real-space terms, where M uses the
    Fourier weights w_i A_i and the real-space terms use (1 - w_i) flux A_i.
    The imaginary part of the inverse transform is asserted to vanish
    (reading R4 makes the product exactly Hermitian)."""
    if not _valid(x, y, flux, r_e, e1, e2):
        img = np.full((W, W), np.nan)
        return (img, None) if return_parts else img
    amp = np.asarray(amp, np.float64)
    a, b, d = covariances(r_e, e1, e2, var, cd)
    w = routing_weights(a, d, W, flags)
    M = galaxy_spectrum(x, y, w * amp, a, b, d, W)
    Ic = inverse_dft2(flux * psf_hat * M)
    scale = max(np.abs(Ic.real).max(), 1e-300)
    if np.abs(Ic.imag).max() > 1e-10 * scale:
        raise AssertionError("inverse transform is not real: Nyquist convention broken")
    I_f = Ic.real
    I_r = real_space_image(x, y, (1.0 - w) * flux * amp, a, b, d, gauss, W)
    if return_parts:
        return I_f + I_r, dict(fourier=I_f, real=I_r, w=w, a=a, b=b, d=d)
    return I_f + I_r


def render_batch(psf, mixtures, gal, flags: int = 0, psf_gauss=None, cd=None, idx=None):
    """Render galaxies `idx` (default all) of a workloads.Galaxies batch.
    Returns a list of float64 stamps (their sizes may differ)."""
    P = np.asarray(psf, np.float64)
    gauss = psf_gauss_moments(P) if psf_gauss is None else np.asarray(psf_gauss, np.float64)
    cache = {}
    out = []
    if idx is None:
        idx = range(len(gal))
    for i in idx:
        p = gal.params(int(i))
        W = p["W"]
        if W not in cache:
            cache[W] = psf_spectrum(P, W)
        amp, var = mixtures.table(p["mix_id"])
        out.append(render_stamp(cache[W], gauss, amp, var, p["x"], p["y"], p["flux"],
                                p["r_e"], p["e1"], p["e2"], W, flags, cd))
    return out
