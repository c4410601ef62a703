"""Pins of the general-Sérsic (interpolated mixture) and composite
(bulge + disk) oracle.

The render is linear in the mixture amplitudes, so interpolation weights and
bulge fractions are pinned exactly by linear combinations of renders at the
grid nodes; node tables reproduce the plain render exactly; off-grid indices
give the invalid (NaN) stamp."""

import numpy as np
import pytest

import oracle as o
from oracle import sersic as osr
import workloads as wl


@pytest.fixture(scope="module")
def setup():
    P = wl.psf_moffat_halo(64)
    return o.psf_spectrum(P, 64), o.psf_gauss_moments(P)


ARGS = (30.6, 33.2, 5.0, 2.2, 0.15, -0.2, 64)


def test_node_index_is_the_node_table(setup):
    S, g = setup
    fam = wl.sersic_family()
    for s in (0, 3, len(fam["n_grid"]) - 1):
        got = osr.render_stamp_sersic(S, g, fam["n_grid"], fam["amp"], fam["var"], float(fam["n_grid"][s]), *ARGS)
        ref = o.render_stamp(S, g, fam["amp"][s].astype(np.float64), fam["var"][s].astype(np.float64), *ARGS)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [0.8, 2.25, 3.9, 5.99])
def test_interpolation_weights_are_linear_in_the_index(setup, n):
    """A family whose variances do not change with n: the stamp is linear in
    the amplitudes, so it is (1 - t) I(n_s) + t I(n_s+1) with t the
    position of n between its two grid neighbours."""
    S, g = setup
    fam = wl.sersic_family()
    grid = fam["n_grid"].astype(np.float64)
    var = np.repeat(fam["var"][4:5].astype(np.float64), len(grid), axis=0)
    amp = fam["amp"].astype(np.float64)
    s = int(np.nonzero(grid <= n)[0][-1])
    t = (n - grid[s]) / (grid[s + 1] - grid[s])
    got = osr.render_stamp_sersic(S, g, grid, amp, var, n, *ARGS)
    lo = o.render_stamp(S, g, amp[s], var[s], *ARGS)
    hi = o.render_stamp(S, g, amp[s + 1], var[s + 1], *ARGS)
    assert np.abs(got - ((1 - t) * lo + t * hi)).max() <= 1e-12 * np.abs(got).max()


def test_off_grid_index_is_invalid(setup):
    S, g = setup
    fam = wl.sersic_family()
    for n in (0.49, 6.01, float("nan")):
        assert np.isnan(osr.render_stamp_sersic(S, g, fam["n_grid"], fam["amp"], fam["var"], n, *ARGS)).all()


@pytest.mark.parametrize("f,rho", [(0.0, 0.5), (1.0, 0.5), (0.3, 0.25), (0.8, 1.0)])
def test_composite_is_the_flux_weighted_sum(setup, f, rho):
    """One-ellipticity composite: (1 - f) disk(r_e) + f bulge(rho r_e)."""
    S, g = setup
    rng = np.random.Generator(np.random.PCG64(3))
    ad, vd = wl.exp6_table(rng)
    ab, vb = wl.dev8_table(rng)
    a, v = osr.composite_mixture(ad, vd, ab, vb, f, rho)
    x, y, F, re, e1, e2, W = ARGS
    got = o.render_stamp(S, g, a, v, x, y, F, re, e1, e2, W)
    disk = o.render_stamp(S, g, ad, vd, x, y, F, re, e1, e2, W)
    bulge = o.render_stamp(S, g, ab, vb, x, y, F, rho * re, e1, e2, W)
    assert np.abs(got - ((1 - f) * disk + f * bulge)).max() <= 1e-12 * np.abs(got).max()


@pytest.mark.parametrize("n,rho", [(0.8, 1.5), (2.25, 0.7), (3.9, 2.0), (5.99, 1.2)])
def test_interpolated_variances_follow_an_r_e_rescaling(setup, n, rho):
    """Variances, pinned by an independent route: a family whose node s+1
    is node s with every variance times rho^2 and the same amplitudes.
    Linear interpolation at t gives variances v_s (1 + t (rho^2 - 1)), and
    since every covariance is v r_e^2 times a matrix of the ellipticity
    (step 3), that stamp is the node-s stamp rendered at
    r_e sqrt(1 + t (rho^2 - 1)).  Any other interpolation rule (geometric,
    or of the standard deviations) renders a different size."""
    S, g = setup
    fam = wl.sersic_family()
    grid = fam["n_grid"].astype(np.float64)
    base_amp = fam["amp"][3].astype(np.float64)
    base_var = fam["var"][3].astype(np.float64)
    steps = np.arange(len(grid), dtype=np.float64)[:, None]
    amp = np.repeat(base_amp[None], len(grid), axis=0)
    var = base_var[None] * rho ** (2.0 * steps)
    s = int(np.nonzero(grid <= n)[0][-1])
    t = (n - grid[s]) / (grid[s + 1] - grid[s])
    x, y, F, re, e1, e2, W = ARGS
    got = osr.render_stamp_sersic(S, g, grid, amp, var, n, *ARGS)
    ref = o.render_stamp(S, g, amp[s], var[s], x, y, F, re * np.sqrt(1.0 + t * (rho * rho - 1.0)), e1, e2, W)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
