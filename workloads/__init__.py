"""Seeded synthetic inputs for the hybrid Fourier-real galaxy-PSF renderer.

This module only draws inputs: mixture tables, pixelized PSFs, galaxy
parameters and request traces.  It holds none of the rendering arithmetic,
so the FP64 oracle and the HIP path can both read identical values from it
without sharing any of the method.

The paper's own inputs (fitted mixture tables of Hogg & Lang 2013, PsfEx PSF
models, Legacy Surveys images) are not available; every generator below is a
stand-in with the shapes and distributions of the paper's workloads.
"""

from .generate import (  # noqa: F401
    SEED_BASE,
    Mixtures,
    Galaxies,
    exp6_table,
    dev8_table,
    mixture_set,
    sersic_family,
    psf_double_gaussian,
    psf_moffat_halo,
    psf_single_gaussian_fit,
    psf_offset_gaussian,
    eigen_psf_moffat,
    draw_galaxies,
    config1,
    config_metric,
    config_eigen,
    config_sersic,
    config_composite,
    config2,
    config3,
    config4_trace,
    config5,
)
