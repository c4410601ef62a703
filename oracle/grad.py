"""FP64 oracle of the render's derivatives (forward-mode, analytic).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The parameters are theta = (x, y, flux, log r_e, e1, e2) per galaxy plus the
mixture amplitudes A_i.  Every derivative image is obtained by differentiating
the steps of Section 2 by hand:

* Fourier path: dI_F/dtheta = Re W^-2 IDFT(flux * P_hat * dM/dtheta), where
  dM/dtheta is the derivative of the Nyquist-averaged mixture transform
  (shift theorem for x, y; Gaussian exponent for the covariances; the routing
  weight w_i for the ramp).
* Real-space path: derivative of the sampled Gaussian N(u; C_i + Sigma_p)
  w.r.t. its centre and covariance, times (1 - w_i), minus dw_i/dtheta times
  the component's real-space image.
* Covariance chain: A = CD^{-1} E with E(r_e, beta(e), theta(e1, e2)) as in
  Section 2 step 3, differentiated through beta and theta (not through the
  trig-free closed form the GPU uses), so the two derivations are independent.

Pinned by central finite differences of the forward oracle (tests), also
with a PSF Gaussian off the centre pixel and with a cross term.
"""

from __future__ import annotations

import math

import numpy as np

from .render import (
    FORCE_FOURIER,
    FORCE_REAL,
    RAMP_LINEAR,
    TWO_PI,
    axis_frequencies,
    covariances,
    inverse_dft2,
    render_stamp,
    _valid,
)

PARAMS = ("x", "y", "flux", "log_re", "e1", "e2")


def _dshape_matrix(r_e, e1, e2, cd=None):
    """E and its derivatives w.r.t. (log r_e, e1, e2), then A = CD^{-1} E."""
    e = math.hypot(e1, e2)
    theta = 0.5 * math.atan2(e2, e1) if e > 0 else 0.0
    beta = (1.0 - e) / (1.0 + e)
    c, s = math.cos(theta), math.sin(theta)
    E = r_e * np.array([[beta * c, s], [-beta * s, c]])
    dE_dbeta = r_e * np.array([[c, 0.0], [-s, 0.0]])
    dE_dtheta = r_e * np.array([[-beta * s, c], [-beta * c, -s]])
    dbeta_de = -2.0 / (1.0 + e) ** 2
    if e > 0:
        de = (e1 / e, e2 / e)
        dth = (-0.5 * e2 / (e * e), 0.5 * e1 / (e * e))
    else:
        de = (0.0, 0.0)
        dth = (0.0, 0.0)
    dE = {
        "log_re": E.copy(),
        "e1": dE_dbeta * dbeta_de * de[0] + dE_dtheta * dth[0],
        "e2": dE_dbeta * dbeta_de * de[1] + dE_dtheta * dth[1],
    }
    Minv = np.eye(2) if cd is None else np.linalg.inv(np.asarray(cd, np.float64).reshape(2, 2))
    A = Minv @ E
    dA = {k: Minv @ v for k, v in dE.items()}
    return A, dA


def _ramp_and_slope(n, flags):
    t = np.clip(n - 3.0, 0.0, 1.0)
    inside = (n > 3.0) & (n < 4.0)
    if flags & FORCE_FOURIER:
        return np.ones_like(n), np.zeros_like(n)
    if flags & FORCE_REAL:
        return np.zeros_like(n), np.zeros_like(n)
    if flags & RAMP_LINEAR:
        return t, np.where(inside, 1.0, 0.0)
    return t * t * (3.0 - 2.0 * t), np.where(inside, 6.0 * t * (1.0 - t), 0.0)


def render_stamp_jacobian(psf_hat, gauss, amp, var, x, y, flux, r_e, e1, e2, W,
                          flags: int = 0, cd=None):
    """Returns (I, J) where J maps each name in PARAMS to dI/dtheta (W x W)
    and "amp" to an array [K, W, W] of dI/dA_i."""
    amp = np.asarray(amp, np.float64)
    var = np.asarray(var, np.float64)
    K = len(amp)
    if not _valid(x, y, flux, r_e, e1, e2):
        nan = np.full((W, W), np.nan)
        return nan, {**{p: nan for p in PARAMS}, "amp": np.full((K, W, W), np.nan)}

    A, dA = _dshape_matrix(r_e, e1, e2, cd)
    B = A @ A.T
    dB = {k: v @ A.T + A @ v.T for k, v in dA.items()}
    a, b, d = covariances(r_e, e1, e2, var, cd)
    n = (W / 2.0) / np.sqrt(a + d)
    w, dw_dn = _ramp_and_slope(n, flags)
    trB = B[0, 0] + B[1, 1]
    # n_i = (W/2) (v_i tr B)^-1/2  ->  dn_i/dtheta = -n_i/2 * dtrB/trB
    dw = {k: dw_dn * (-0.5 * n * (v[0, 0] + v[1, 1]) / trB) for k, v in dB.items()}

    # ---- Fourier path ----------------------------------------------------
    lo, hi = axis_frequencies(W)
    reps = [np.meshgrid(fx, fy) for fx in (lo, hi) for fy in (lo, hi)]
    dM = {p: np.zeros((W, W), np.complex128) for p in PARAMS}
    M = np.zeros((W, W), np.complex128)
    dM_amp = np.zeros((K, W, W), np.complex128)
    for NU, OM in reps:
        phase = np.exp(-1j * TWO_PI * (x * NU + y * OM))
        S = np.zeros((W, W))
        dS = {k: np.zeros((W, W)) for k in dB}
        for i in range(K):
            g = np.exp(-2.0 * math.pi**2 * (a[i] * NU * NU + 2 * b[i] * NU * OM + d[i] * OM * OM))
            S += w[i] * amp[i] * g
            dM_amp[i] += phase * w[i] * g
            for k, dBk in dB.items():
                dq = -2.0 * math.pi**2 * var[i] * (dBk[0, 0] * NU * NU + 2 * dBk[0, 1] * NU * OM
                                                   + dBk[1, 1] * OM * OM)
                dS[k] += amp[i] * g * (w[i] * dq + dw[k][i])
        M += phase * S
        dM["x"] += -1j * TWO_PI * NU * phase * S
        dM["y"] += -1j * TWO_PI * OM * phase * S
        for k in dS:
            dM[k] += phase * dS[k]
    M /= 4.0
    dM_amp /= 4.0
    for p in dM:
        dM[p] /= 4.0

    def to_img(spec):
        return inverse_dft2(flux * psf_hat * spec).real

    I_f = to_img(M)
    J = {p: to_img(dM[p]) for p in ("x", "y", "log_re", "e1", "e2")}
    J_amp = np.stack([to_img(dM_amp[i]) for i in range(K)]) if K else np.zeros((0, W, W))

    # ---- real-space path ---------------------------------------------------
    mux, muy, pxx, pxy, pyy, pamp = [float(v) for v in gauss]
    yy, xx = np.mgrid[0:W, 0:W].astype(np.float64)
    ux = xx - x - mux
    uy = yy - y - muy
    I_r = np.zeros((W, W))
    for i in range(K):
        r = 1.0 - w[i]
        if r == 0.0 and all(dw[k][i] == 0.0 for k in dw):
            continue
        sxx, sxy, syy = a[i] + pxx, b[i] + pxy, d[i] + pyy
        det = sxx * syy - sxy * sxy
        ixx, ixy, iyy = syy / det, -sxy / det, sxx / det
        zx = ixx * ux + ixy * uy      # (Sigma^-1 u)_x
        zy = ixy * ux + iyy * uy
        N = np.exp(-0.5 * (ux * zx + uy * zy)) / (TWO_PI * math.sqrt(det))
        unit = flux * amp[i] * pamp * N
        I_r += r * unit
        J["x"] += r * unit * zx
        J["y"] += r * unit * zy
        J_amp[i] += r * flux * pamp * N
        for k, dBk in dB.items():
            dSxx, dSxy, dSyy = var[i] * dBk[0, 0], var[i] * dBk[0, 1], var[i] * dBk[1, 1]
            # dN = N [ z^T dSigma z / 2 - tr(Sigma^-1 dSigma) / 2 ]
            quad = zx * zx * dSxx + 2 * zx * zy * dSxy + zy * zy * dSyy
            tr = ixx * dSxx + 2 * ixy * dSxy + iyy * dSyy
            J[k] += r * unit * 0.5 * (quad - tr) - dw[k][i] * unit

    I = I_f + I_r
    J["flux"] = I / flux if flux != 0 else np.zeros_like(I)
    J["amp"] = J_amp
    return I, J


def loss_gradient(g, J):
    """dL/dtheta = sum_pixels g * dI/dtheta for each parameter; amplitudes
    give an array of K values."""
    out = {p: float(np.sum(g * J[p])) for p in PARAMS}
    out["amp"] = np.tensordot(J["amp"], g, axes=([1, 2], [0, 1]))
    return out


def fd_gradient(psf_hat, gauss, amp, var, params, W, g, flags=0, h=1e-3, cd=None):
    """Central finite differences of L = sum(g * I) in FP64 with step h on
    x, y, log r_e, e1, e2 and the amplitudes, and a relative step on flux."""
    amp = np.asarray(amp, np.float64)

    def L(pp, aa):
        img = render_stamp(psf_hat, gauss, aa, var, pp["x"], pp["y"], pp["flux"],
                           pp["r_e"], pp["e1"], pp["e2"], W, flags, cd)
        return float(np.sum(g * img))

    out = {}
    for p in PARAMS:
        up, dn = dict(params), dict(params)
        if p == "log_re":
            up["r_e"] = params["r_e"] * math.exp(h)
            dn["r_e"] = params["r_e"] * math.exp(-h)
            step = h
        elif p == "flux":
            step = h * params["flux"]
            up["flux"] += step
            dn["flux"] -= step
        else:
            up[p] += h
            dn[p] -= h
            step = h
        out[p] = (L(up, amp) - L(dn, amp)) / (2 * step)
    ga = np.zeros(len(amp))
    for i in range(len(amp)):
        au, ad = amp.copy(), amp.copy()
        au[i] += h
        ad[i] -= h
        ga[i] = (L(params, au) - L(params, ad)) / (2 * h)
    out["amp"] = ga
    return out
