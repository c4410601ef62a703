"""FP64 oracle of the Lanczos sub-pixel shift (Lang 2020, Section 2, step 8:
the optional alternative to the Fourier phase, in which the stamp is rendered
at the integer part of the galaxy position and the finished pixel stamp,
real-space terms included, is shifted by the fractional part with Lanczos
interpolation; Section 2 also notes that this route brings tiny galaxies
closer to point sources).

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark's checks; never
by the product path.

Readings (the paper gives no order, normalisation or edge rule):
  L1  Order 3: L(t) = sinc(t) sinc(t/3) for |t| < 3, else 0, with
      sinc(t) = sin(pi t) / (pi t).
  L2  Shift by the fractional part f = x - floor(x) in [0, 1) per axis:
      out[c] = sum_{d=-3..2} w_d in[c + d],  w_d = L(d + f) / sum_d' L(d' + f)
      (the interpolated value of the input at c - f; the six weights are
      normalised to unit sum so a constant is kept exactly).
  L3  Separable: the same rule along rows and along columns.
  L4  Pixels outside the stamp count as zero (the stamp is not periodic in
      pixel space).
  L5  The Fourier part then carries no fractional phase, and the real-space
      components are centred on the integer position too.
"""

from __future__ import annotations

import math

import numpy as np

from .render import render_stamp

LANCZOS3 = 8
TAPS = np.arange(-3, 3)  # d = -3 .. 2


def lanczos3(t: float) -> float:
    """Reading L1."""
    t = float(t)
    if t == 0.0:
        return 1.0
    if abs(t) >= 3.0 or t == round(t):  # sinc vanishes exactly at the other integers
        return 0.0
    a = math.pi * t
    return (math.sin(a) / a) * (math.sin(a / 3.0) / (a / 3.0))


def lanczos_weights(f: float) -> np.ndarray:
    """Reading L2: the six normalised weights for taps d = -3..2."""
    w = np.array([lanczos3(d + f) for d in TAPS], np.float64)
    return w / w.sum()


def lanczos_shift(img: np.ndarray, fx: float, fy: float) -> np.ndarray:
    """Readings L2-L4: separable shift of a stamp by (fx, fy) in [0, 1)^2."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    wx, wy = lanczos_weights(fx), lanczos_weights(fy)
    pad = np.zeros((H, W + 6))
    pad[:, 3:W + 3] = img
    rows = np.zeros((H, W))
    for k, d in enumerate(TAPS):
        rows += wx[k] * pad[:, 3 + d:3 + d + W]  # rows[r, c] += w_d in[r, c + d]
    pad = np.zeros((H + 6, W))
    pad[3:H + 3, :] = rows
    out = np.zeros((H, W))
    for k, d in enumerate(TAPS):
        out += wy[k] * pad[3 + d:3 + d + H, :]
    return out


def render_stamp_lanczos(psf_hat, gauss, amp, var, x, y, flux, r_e, e1, e2, W, flags: int = 0, cd=None):
    """Steps 3-8 with the Lanczos sub-pixel shift (reading L5): the stamp at
    (floor x, floor y), shifted by the fractional parts."""
    if not all(math.isfinite(v) for v in (x, y)):
        return np.full((W, W), np.nan)
    xi, yi = math.floor(x), math.floor(y)
    img = render_stamp(psf_hat, gauss, amp, var, float(xi), float(yi), flux, r_e, e1, e2, W, flags, cd)
    return lanczos_shift(img, x - xi, y - yi)
