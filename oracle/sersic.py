"""FP64 oracle of general-Sérsic and composite (bulge + disk) galaxies
(Lang 2020: Section 1 on the profile family and its bulge-disk combinations,
and the closing discussion that mixture amplitudes and variances vary
smoothly with the Sérsic index, so tables fitted on a grid of indices can be
interpolated at the same per-galaxy cost).

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark's checks; never
by the product path.

The fitted tables are not available; the workloads generator provides smooth
synthetic ones.  Readings:
  S1  Interpolation is piecewise linear in the index n, per component, of the
      amplitude and of the variance, between the two grid indices around n;
      the grid tables share one component count K (components correspond
      across the grid).
  S2  n outside [n_0, n_last] or not finite is an invalid galaxy (NaN stamp,
      as reading R8).
  S3  A composite galaxy with one ellipticity is one mixture: disk components
      with amplitudes (1 - f) A_d and variances v_d, bulge components with
      amplitudes f A_b and variances rho^2 v_b, where f is the bulge flux
      fraction and rho = r_e(bulge) / r_e(disk); the galaxy's r_e is the
      disk's.  Bulges and disks with different ellipticities are the sum of
      two renders (the library's accumulate flag).
"""

from __future__ import annotations

import math

import numpy as np

from .render import psf_spectrum, psf_gauss_moments, render_stamp


def sersic_mixture(n_grid, amp, var, n: float):
    """Reading S1: (A_k(n), v_k(n)), or None when n is off the grid (S2).
    Pinned by linearity in the amplitudes and, for the variances, by a
    family whose nodes differ by a common variance factor, which must
    render as the node stamp at a rescaled r_e (tests)."""
    n_grid = np.asarray(n_grid, np.float64)
    amp = np.asarray(amp, np.float64)
    var = np.asarray(var, np.float64)
    if not math.isfinite(n) or n < n_grid[0] or n > n_grid[-1]:
        return None
    s = int(np.searchsorted(n_grid, n, side="right")) - 1
    s = min(max(s, 0), len(n_grid) - 2)
    t = (n - n_grid[s]) / (n_grid[s + 1] - n_grid[s])
    return (1.0 - t) * amp[s] + t * amp[s + 1], (1.0 - t) * var[s] + t * var[s + 1]


def composite_mixture(amp_d, var_d, amp_b, var_b, f: float, rho: float):
    """Reading S3: the concatenated mixture of a one-ellipticity composite."""
    a = np.concatenate([(1.0 - f) * np.asarray(amp_d, np.float64), f * np.asarray(amp_b, np.float64)])
    v = np.concatenate([np.asarray(var_d, np.float64), rho * rho * np.asarray(var_b, np.float64)])
    return a, v


def render_stamp_sersic(psf_hat, gauss, n_grid, amp, var, n, x, y, flux, r_e, e1, e2, W, flags: int = 0):
    m = sersic_mixture(n_grid, amp, var, n)
    if m is None:
        return np.full((W, W), np.nan)
    return render_stamp(psf_hat, gauss, m[0], m[1], x, y, flux, r_e, e1, e2, W, flags)


def render_batch_sersic(psf, family, gal, sersic_n, flags: int = 0, idx=None):
    """Render galaxies `idx` of a workloads.Galaxies batch with a Sérsic
    family dict(n_grid, amp [S][K], var [S][K]) and per-galaxy indices."""
    P = np.asarray(psf, np.float64)
    gauss = psf_gauss_moments(P)
    cache, out = {}, []
    if idx is None:
        idx = range(len(gal))
    for i in idx:
        p = gal.params(int(i))
        W = p["W"]
        if W not in cache:
            cache[W] = psf_spectrum(P, W)
        out.append(render_stamp_sersic(cache[W], gauss, family["n_grid"], family["amp"], family["var"],
                                       float(sersic_n[i]), p["x"], p["y"], p["flux"], p["r_e"], p["e1"],
                                       p["e2"], W, flags))
    return out
