"""FP64 oracle of the spatially varying (eigen-)PSF render (Lang 2020,
Section 2, the step-2 discussion of PSF models whose pixelized components
carry polynomial amplitudes over the image).

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark's checks; never
by the product path.

The PSF at image position (X, Y) is the pixel-space sum of J component images
weighted by polynomials of the normalised position, and the stamp is then the
ordinary render with that PSF (steps 2-8 of render.py).  The paper's point is
that the same sum can be taken over the components' Fourier transforms; the
oracle takes it in pixel space, before the transform, so the GPU path (which
sums transforms) is checked against an independent route.

Readings:
  E1  Normalised coordinates u = (X - x_off) / x_scale, v = (Y - y_off) / y_scale.
  E2  Polynomial terms u^a v^b with a + b <= degree, ordered by the power of
      v, then the power of u: 1, u, u^2, ..., v, u v, ..., v^degree (the
      order PSF-modelling tools such as PsfEx use).
  E3  Component weights c_j = sum_t coef[j, t] term_t(u, v).
  E4  The real-space PSF Gaussian of a varying PSF is the moment Gaussian of
      the PSF at that position (reading R6 applied to the summed image).
"""

from __future__ import annotations

import numpy as np

from .render import psf_gauss_moments, psf_spectrum, render_stamp


def poly_exponents(degree: int):
    """(a, b) of each term u^a v^b in the order of reading E2."""
    return [(a, b) for b in range(degree + 1) for a in range(degree + 1 - b)]


def poly_terms(u: float, v: float, degree: int) -> np.ndarray:
    return np.array([u**a * v**b for a, b in poly_exponents(degree)], np.float64)


def eigen_weights(coef, degree: int, norm, X: float, Y: float) -> np.ndarray:
    """Readings E1-E3: c_j at image position (X, Y)."""
    coef = np.asarray(coef, np.float64)
    u = (X - norm[0]) / norm[1]
    v = (Y - norm[2]) / norm[3]
    return coef @ poly_terms(u, v, degree)


def eigen_psf_image(comps, coef, degree: int, norm, X: float, Y: float) -> np.ndarray:
    """The pixelized PSF at (X, Y): sum_j c_j comps[j]."""
    c = eigen_weights(coef, degree, norm, X, Y)
    return np.tensordot(c, np.asarray(comps, np.float64), axes=1)


def render_stamp_eigen(comps, coef, degree, norm, X, Y, amp, var, x, y, flux, r_e, e1, e2, W,
                       flags: int = 0, cd=None):
    """Steps 2-8 with the PSF evaluated at image position (X, Y)."""
    P = eigen_psf_image(comps, coef, degree, norm, X, Y)
    return render_stamp(psf_spectrum(P, W), psf_gauss_moments(P), amp, var, x, y, flux, r_e, e1, e2,
                        W, flags, cd)


def render_batch_eigen(eig, mixtures, gal, psf_x, psf_y, flags: int = 0, idx=None):
    """Render galaxies `idx` (default all) of a workloads.Galaxies batch with
    an eigen-PSF description `eig` (dict with comps, coef, degree, norm)."""
    out = []
    if idx is None:
        idx = range(len(gal))
    for i in idx:
        p = gal.params(int(i))
        amp, var = mixtures.table(p["mix_id"])
        out.append(render_stamp_eigen(eig["comps"], eig["coef"], eig["degree"], eig["norm"],
                                      float(psf_x[i]), float(psf_y[i]), amp, var, p["x"], p["y"],
                                      p["flux"], p["r_e"], p["e1"], p["e2"], p["W"], flags))
    return out
