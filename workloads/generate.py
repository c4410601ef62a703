"""Seeded input generators (NumPy PCG64).  No rendering arithmetic lives here.

Conventions shared with the renderer's public interface:

* A pixel at (row r, column c) has its centre at (x = c, y = r), 0-based.
* A pixelized PSF of shape (S_y, S_x) has its centre at pixel (S_y/2, S_x/2).
* A galaxy is (x, y, flux, r_e, e1, e2, mix_id); r_e is in pixels.
* A mixture table t has K[t] components with amplitudes amp[t, :K[t]] and
  isotropic variances var[t, :K[t]] in units of r_e^2.

Every generator takes the config's seed and is deterministic.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2012157970
KMAX = 16


# --------------------------------------------------------------------------
# Mixture tables.  The fitted exponential / deVaucouleurs tables are not
# available, so amplitudes are drawn from Dirichlet(1) and variances are
# log-spaced, as the workload descriptions prescribe.
# --------------------------------------------------------------------------

def exp6_table(rng: np.random.Generator):
    """Exponential-like stand-in: K=6, amplitudes ~ Dirichlet(1), variances
    log-spaced over [1e-3, 3] (r_e^2 units)."""
    amp = rng.dirichlet(np.ones(6))
    var = np.logspace(math.log10(1e-3), math.log10(3.0), 6)
    return amp, var


def dev8_table(rng: np.random.Generator):
    """deVaucouleurs-like stand-in: K=8, amplitudes ~ Dirichlet(1), variances
    log-spaced over [1e-4, 10] (r_e^2 units)."""
    amp = rng.dirichlet(np.ones(8))
    var = np.logspace(math.log10(1e-4), math.log10(10.0), 8)
    return amp, var


@dataclasses.dataclass
class Mixtures:
    """A set of mixture tables, padded to KMAX columns (padding is zero)."""

    K: np.ndarray          # int32 [n_tables]
    amp: np.ndarray        # float64 [n_tables, KMAX]
    var: np.ndarray        # float64 [n_tables, KMAX]

    @property
    def n_tables(self) -> int:
        return int(self.K.shape[0])

    def table(self, t: int):
        k = int(self.K[t])
        return self.amp[t, :k].copy(), self.var[t, :k].copy()

    def as_f32(self) -> "Mixtures":
        return Mixtures(self.K.astype(np.int32),
                        self.amp.astype(np.float32).astype(np.float64),
                        self.var.astype(np.float32).astype(np.float64))


def sersic_family(K: int = 8, n_grid=None):
    """Synthetic Sérsic mixture family: K components per grid index n whose
    amplitudes (unit sum) and variances (r_e^2 units) vary smoothly with n,
    shaped like the fitted families the paper describes (larger n: more
    weight at both the smallest and the largest variances).  The fitted
    tables of the paper are not available.  Returns dict(n_grid [S],
    amp [S][K], var [S][K]) float32."""
    n_grid = np.arange(0.5, 6.01, 0.5) if n_grid is None else np.asarray(n_grid, np.float64)
    k = np.arange(K, dtype=np.float64)
    amp, var = [], []
    for n in n_grid:
        lo = -2.0 - 0.45 * (n - 1.0)          # log10 of the smallest variance
        hi = 0.15 + 0.11 * n                   # log10 of the largest variance
        var.append(10.0 ** (lo + (hi - lo) * k / (K - 1)))
        centre = (K - 1) * (0.62 - 0.05 * n)
        width = 1.2 + 0.35 * n
        a = np.exp(-0.5 * ((k - centre) / width) ** 2) + 0.02 * n * np.exp(-k)
        amp.append(a / a.sum())
    return dict(n_grid=n_grid.astype(np.float32), amp=np.array(amp, np.float32), var=np.array(var, np.float32))


def mixture_set(tables) -> Mixtures:
    n = len(tables)
    K = np.zeros(n, np.int32)
    amp = np.zeros((n, KMAX))
    var = np.zeros((n, KMAX))
    for t, (a, v) in enumerate(tables):
        k = len(a)
        assert k <= KMAX and len(v) == k
        K[t] = k
        amp[t, :k] = a
        var[t, :k] = v
    return Mixtures(K, amp, var)


# --------------------------------------------------------------------------
# PSFs: pixel grids sampled at pixel centres about (S/2, S/2), normalised to
# unit sum.  Each profile component is normalised to unit integral first.
# --------------------------------------------------------------------------

def _grid(S: int):
    r = np.arange(S, dtype=np.float64) - S // 2
    X, Y = np.meshgrid(r, r)  # X varies along columns (x), Y along rows (y)
    return X, Y


def _gauss_profile(X, Y, sigma):
    return np.exp(-0.5 * (X * X + Y * Y) / sigma**2) / (2 * math.pi * sigma**2)


def _moffat_profile(X, Y, fwhm, beta):
    alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    norm = (beta - 1.0) / (math.pi * alpha**2)
    return norm * (1.0 + (X * X + Y * Y) / alpha**2) ** (-beta)


def psf_double_gaussian(S: int = 64, sigmas=(1.7, 4.0), weights=(0.9, 0.1)):
    """Double-Gaussian PSF: sum_j w_j N(0, s_j^2 I) sampled on S x S pixels."""
    X, Y = _grid(S)
    p = sum(w * _gauss_profile(X, Y, s) for w, s in zip(weights, sigmas))
    return p / p.sum()


def psf_moffat_halo(S: int = 64, fwhm: float = 4.5, beta: float = 3.0,
                    halo_sigma: float = 8.0, halo_weight: float = 0.01):
    """Moffat core plus a broad Gaussian halo, sampled on S x S pixels."""
    X, Y = _grid(S)
    p = ((1.0 - halo_weight) * _moffat_profile(X, Y, fwhm, beta)
         + halo_weight * _gauss_profile(X, Y, halo_sigma))
    return p / p.sum()


OFFSET_PSF_MU = (0.37, -0.21)
OFFSET_PSF_COV = ((3.1, 0.8), (0.8, 2.2))


def psf_offset_gaussian(S: int = 64, mu=OFFSET_PSF_MU, cov=OFFSET_PSF_COV):
    """One elliptical Gaussian N(mu, cov) sampled on S x S pixels, mu measured
    from the centre pixel (S/2, S/2) and off it, cov with a cross term.
    Returns (pixels normalised to unit sum, the explicit single-Gaussian
    description {mu_x, mu_y, c_xx, c_xy, c_yy, amp = 1}).  At these widths the
    sampled grid's moments equal (mu, cov) to ~1e-15, so the description is
    exact for the pixel PSF: a test PSF for the real-space route's mean and
    cross term, which centred isotropic PSFs leave untested."""
    X, Y = _grid(S)
    (cxx, cxy), (_, cyy) = cov
    det = cxx * cyy - cxy * cxy
    ux, uy = X - mu[0], Y - mu[1]
    p = np.exp(-0.5 * (cyy * ux * ux - 2.0 * cxy * ux * uy + cxx * uy * uy) / det)
    return p / p.sum(), np.array([mu[0], mu[1], cxx, cxy, cyy, 1.0])


def eigen_psf_moffat(S: int = 64, degree: int = 2, image_size: float = 4096.0, n_fit: int = 7):
    """Synthetic spatially varying PSF in eigen form (components with
    polynomial amplitudes, as PSF-modelling tools produce them).  The true
    PSF is a Moffat (beta = 3) whose FWHM and ellipticity drift smoothly
    over an image_size x image_size field, plus a 1% Gaussian halo.  As such
    tools do, one component image per polynomial term is fitted by least
    squares, pixel by pixel, to PSFs sampled on an n_fit x n_fit grid of
    positions.  Returns dict(comps [T][S][S] float32, coef [T][T] (identity),
    degree, norm (x_off, x_scale, y_off, y_scale))."""
    X, Y = _grid(S)
    half = image_size / 2.0
    grid = np.linspace(-1.0, 1.0, n_fit)
    exps = [(a, b) for b in range(degree + 1) for a in range(degree + 1 - b)]
    rows, imgs = [], []
    for v in grid:
        for u in grid:
            fwhm = 4.5 + 0.4 * u - 0.3 * v + 0.15 * u * v + 0.2 * u * u - 0.1 * v * v
            q = 1.0 - 0.06 * (u + 0.5 * v)          # axis ratio
            ang = 0.4 * u - 0.3 * v                  # position angle
            c, s_ = math.cos(ang), math.sin(ang)
            Xr, Yr = c * X + s_ * Y, (-s_ * X + c * Y) / q
            p = 0.99 * _moffat_profile(Xr, Yr, fwhm, 3.0) + 0.01 * _gauss_profile(X, Y, 8.0)
            imgs.append((p / p.sum()).ravel())
            rows.append([u**a * v**b for a, b in exps])
    A = np.array(rows)
    comps, *_ = np.linalg.lstsq(A, np.array(imgs), rcond=None)
    T = len(exps)
    return dict(comps=comps.reshape(T, S, S).astype(np.float32), coef=np.eye(T), degree=degree,
                norm=np.array([half, half, half, half]))


def psf_single_gaussian_fit(P: np.ndarray) -> np.ndarray:
    """Least-squares fit of one centred isotropic Gaussian (variance, amplitude)
    to the PSF pixels.  Returns {mu_x, mu_y, c_xx, c_xy, c_yy, amp} in the
    renderer's convention (offsets from the PSF centre pixel).

    This is input preparation: the paper leaves the way the single-Gaussian
    PSF approximation is obtained unstated, so the fit is made once here and
    handed to every renderer as an explicit input."""
    from scipy.optimize import least_squares

    S = P.shape[0]
    X, Y = _grid(S)
    R2 = X * X + Y * Y

    def resid(p):
        var, amp = math.exp(p[0]), p[1]
        return (amp * np.exp(-0.5 * R2 / var) / (2 * math.pi * var) - P).ravel()

    sol = least_squares(resid, x0=[math.log(4.0), 1.0], xtol=1e-14, ftol=1e-14)
    var, amp = math.exp(sol.x[0]), float(sol.x[1])
    return np.array([0.0, 0.0, var, 0.0, var, amp])


# --------------------------------------------------------------------------
# Galaxy parameters.
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Galaxies:
    """Structure-of-arrays galaxy parameters (float32 as handed to the GPU)."""

    x: np.ndarray
    y: np.ndarray
    flux: np.ndarray
    r_e: np.ndarray
    e1: np.ndarray
    e2: np.ndarray
    mix_id: np.ndarray     # int32
    W: np.ndarray          # int32 stamp size per galaxy

    def __len__(self):
        return int(self.x.shape[0])

    def subset(self, idx) -> "Galaxies":
        return Galaxies(*(getattr(self, f.name)[idx] for f in dataclasses.fields(self)))

    def params(self, i: int):
        return dict(x=float(self.x[i]), y=float(self.y[i]), flux=float(self.flux[i]),
                    r_e=float(self.r_e[i]), e1=float(self.e1[i]), e2=float(self.e2[i]),
                    mix_id=int(self.mix_id[i]), W=int(self.W[i]))


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def _ellipticities(rng, n, sigma=0.2, emax=0.7):
    e1 = rng.normal(0.0, sigma, n)
    e2 = rng.normal(0.0, sigma, n)
    e = np.hypot(e1, e2)
    big = e >= emax
    scale = np.where(big, 0.699 / np.maximum(e, 1e-300), 1.0)
    return e1 * scale, e2 * scale


def draw_galaxies(rng, n, W, mix_id, r_e_range=(0.5, 8.0), flux_range=(1.0, 1e4)):
    """Galaxy draws with the batched-render distributions: r_e log-uniform,
    e1, e2 ~ N(0, 0.2) rescaled to 0.699 when |e| >= 0.7, flux log-uniform,
    centre at (W/2, W/2) plus a uniform sub-pixel offset in [0, 1)^2."""
    W = np.broadcast_to(np.asarray(W, np.int32), (n,)).copy()
    mix_id = np.broadcast_to(np.asarray(mix_id, np.int32), (n,)).copy()
    r_e = _log_uniform(rng, *r_e_range, n)
    e1, e2 = _ellipticities(rng, n)
    flux = _log_uniform(rng, *flux_range, n)
    dx = rng.uniform(0.0, 1.0, n)
    dy = rng.uniform(0.0, 1.0, n)
    x = W / 2 + dx
    y = W / 2 + dy
    f32 = lambda a: np.asarray(a, np.float32)
    return Galaxies(f32(x), f32(y), f32(flux), f32(r_e), f32(e1), f32(e2), mix_id, W)


# --------------------------------------------------------------------------
# Configurations.
# --------------------------------------------------------------------------

FORCE_FOURIER, FORCE_REAL, RAMP_LINEAR = 1, 2, 4


def config1():
    """Tiny case: one EXP6 galaxy (r_e=3, e=(0.2,-0.1), flux 1) rendered into a
    64x64 stamp at the 16 sub-pixel offsets {0,.25,.5,.75}^2 about (32,32),
    double-Gaussian PSF in FP64, every component in Fourier space."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 1))
    mix = mixture_set([exp6_table(rng)])
    psf = psf_double_gaussian(64)
    offs = np.array([0.0, 0.25, 0.5, 0.75])
    dx, dy = np.meshgrid(offs, offs)
    n = 16
    gal = Galaxies(
        x=(32.0 + dx.ravel()).astype(np.float32), y=(32.0 + dy.ravel()).astype(np.float32),
        flux=np.ones(n, np.float32), r_e=np.full(n, 3.0, np.float32),
        e1=np.full(n, 0.2, np.float32), e2=np.full(n, -0.1, np.float32),
        mix_id=np.zeros(n, np.int32), W=np.full(n, 64, np.int32))
    return dict(name="tiny-64-exp6-16offsets", mix=mix, psf=psf, psf_gauss=None,
                gal=gal, flags=FORCE_FOURIER)


def _psf_b():
    return psf_moffat_halo(64, fwhm=4.5, beta=3.0, halo_sigma=8.0, halo_weight=0.01)


def config_metric(n=100_000):
    """Throughput workload: n DEV8 galaxies in 64x64 stamps, Moffat+halo PSF,
    batched-render parameter distributions, hybrid routing on."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2))
    dev = dev8_table(rng)
    mix = mixture_set([dev])
    gal = draw_galaxies(rng, n, 64, 0)
    return dict(name="dev8-64x64-moffat", mix=mix, psf=_psf_b().astype(np.float32),
                psf_gauss=None, gal=gal, flags=0)


def config_eigen(n=100_000):
    """The throughput workload with a spatially varying PSF: n DEV8 galaxies
    in 64x64 stamps at uniform positions over a 4096 x 4096 image, each
    rendered with the eigen-PSF evaluated at its position."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 6))
    dev = dev8_table(rng)
    mix = mixture_set([dev])
    gal = draw_galaxies(rng, n, 64, 0)
    psf_x = rng.uniform(0.0, 4096.0, n).astype(np.float32)
    psf_y = rng.uniform(0.0, 4096.0, n).astype(np.float32)
    return dict(name="dev8-64x64-eigenpsf", mix=mix, eig=eigen_psf_moffat(64, 2), gal=gal,
                psf_x=psf_x, psf_y=psf_y, flags=0)


def config_sersic(n=100_000):
    """General-Sérsic throughput workload: n galaxies in 64x64 stamps with the
    metric workload's parameter distributions and a Sérsic index uniform on
    [0.5, 6], rendered with the synthetic Sérsic family (K = 8)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7))
    gal = draw_galaxies(rng, n, 64, 0)
    sersic_n = rng.uniform(0.5, 6.0, n).astype(np.float32)
    return dict(name="sersic8-64x64-moffat", family=sersic_family(8), psf=_psf_b().astype(np.float32),
                gal=gal, sersic_n=sersic_n, flags=0)


def config_composite(n=100_000):
    """Bulge + disk workload: EXP6 disks and DEV8 bulges sharing an
    ellipticity, bulge fraction uniform on [0, 1], bulge-to-disk radius ratio
    log-uniform on [0.2, 1]; 64x64 stamps."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 8))
    disk = exp6_table(rng)
    bulge = dev8_table(rng)
    gal = draw_galaxies(rng, n, 64, 0)
    frac = rng.uniform(0.0, 1.0, n).astype(np.float32)
    rho = _log_uniform(rng, 0.2, 1.0, n).astype(np.float32)
    return dict(name="composite-exp6-dev8-64x64", mix=mixture_set([disk, bulge]), psf=_psf_b().astype(np.float32),
                gal=gal, bulge_frac=frac, bulge_rho=rho, flags=0)


def config2(n=100_000):
    """Mixed batch: half EXP6 (table 0), half DEV8 (table 1); stamps 32/64/128
    in a 5:4:1 mix; Moffat+halo PSF."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 2))
    mix = mixture_set([exp6_table(rng), dev8_table(rng)])
    mix_id = (np.arange(n) % 2).astype(np.int32)
    W = rng.choice(np.array([32, 64, 128], np.int32), size=n, p=[0.5, 0.4, 0.1])
    gal = draw_galaxies(rng, n, W, mix_id)
    return dict(name="mixed-32-64-128", mix=mix, psf=_psf_b().astype(np.float32),
                psf_gauss=None, gal=gal, flags=0)


def config3(n=20_000):
    """Large galaxies: r_e log-uniform 10..60 px, DEV8, stamps 128 and 256
    equally, double-Gaussian PSF (core FWHM 4 px) in FP32 with its fitted
    single-Gaussian approximation."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 3))
    mix = mixture_set([dev8_table(rng)])
    W = rng.choice(np.array([128, 256], np.int32), size=n)
    gal = draw_galaxies(rng, n, W, 0, r_e_range=(10.0, 60.0))
    psf = psf_double_gaussian(64).astype(np.float32)
    gauss = psf_single_gaussian_fit(psf.astype(np.float64))
    return dict(name="large-128-256", mix=mix, psf=psf, psf_gauss=gauss, gal=gal, flags=0)


def config4_trace(duration_s=60.0, rate_hz=2000.0, n_psf=64, seed_offset=4, restricted=False):
    """Serving trace: Poisson arrivals; each request has 1..4096 galaxies
    (log-uniform), one of n_psf resident PSFs (Moffat+halo, FWHM uniform
    3..7 px) and a stamp size from {16, 32, 64, 128, 256}.  Galaxy parameters
    are drawn per request with the batched-render distributions.

    restricted=True gives the variant tied to the throughput workload: every
    request uses 64x64 stamps, the DEV8 table and the throughput workload's
    Moffat+halo PSF."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))
    if restricted:
        mix = mixture_set([dev8_table(np.random.Generator(np.random.PCG64(SEED_BASE + 2)))])
        psfs = [_psf_b().astype(np.float32)]
        sizes, tables = [64], [0]
    else:
        mix = mixture_set([exp6_table(rng), dev8_table(rng)])
        fwhm = rng.uniform(3.0, 7.0, n_psf)
        psfs = [psf_moffat_halo(64, fwhm=float(f)).astype(np.float32) for f in fwhm]
        sizes, tables = [16, 32, 64, 128, 256], [0, 1]
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        n = int(min(4096, max(1, math.floor(_log_uniform(rng, 1.0, 4097.0, 1)[0]))))
        W = int(rng.choice(sizes))
        p = int(rng.integers(0, len(psfs)))
        gal = draw_galaxies(rng, n, W, int(rng.choice(tables)))
        reqs.append(dict(t=t, psf=p, W=W, gal=gal))
    return dict(name="serving-trace" + ("-64" if restricted else ""), mix=mix, psfs=psfs, requests=reqs)


def config5(n=10_000):
    """Differentiation workload: n DEV8 galaxies in 64x64 stamps, Moffat+halo
    PSF, plus perturbed parameters for the fit target (dx, dy ~ N(0, 0.1) px,
    d log r_e ~ N(0, 0.05), de ~ N(0, 0.02) re-clipped, dF/F ~ N(0, 0.05)) and
    a unit-normal noise field the caller scales by 0.01 x peak."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 5))
    mix = mixture_set([dev8_table(rng)])
    gal = draw_galaxies(rng, n, 64, 0)
    f32 = lambda a: np.asarray(a, np.float32)
    pe1 = gal.e1 + rng.normal(0, 0.02, n)
    pe2 = gal.e2 + rng.normal(0, 0.02, n)
    e = np.hypot(pe1, pe2)
    s = np.where(e >= 0.7, 0.699 / np.maximum(e, 1e-300), 1.0)
    pert = Galaxies(
        x=f32(gal.x + rng.normal(0, 0.1, n)), y=f32(gal.y + rng.normal(0, 0.1, n)),
        flux=f32(gal.flux * (1 + rng.normal(0, 0.05, n))),
        r_e=f32(gal.r_e * np.exp(rng.normal(0, 0.05, n))),
        e1=f32(pe1 * s), e2=f32(pe2 * s), mix_id=gal.mix_id.copy(), W=gal.W.copy())
    noise_seed = SEED_BASE + 50
    return dict(name="grad-dev8-64x64", mix=mix, psf=_psf_b().astype(np.float32),
                psf_gauss=None, gal=gal, target_gal=pert, noise_seed=noise_seed, flags=0)


def noise_field(seed, n, W):
    """Unit-normal noise, float32 [n, W, W]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, W, W), dtype=np.float32)
