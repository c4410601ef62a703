"""MI355X (gfx950) renderer for the hybrid Fourier-real mixture-of-Gaussians
galaxy-PSF convolution (Lang 2020, arXiv:2012.15797).

The computation lives in libgfc.so (HIP kernels behind the C ABI of
include/gfc.h); this package only marshals arguments to it, with torch
supplying device memory and streams.  There is no CPU fallback: when the
library is missing, loading it raises.
"""

from ._lib import (  # noqa: F401
    GFC_ACCUMULATE,
    GFC_FORCE_FOURIER,
    GFC_FORCE_REAL,
    GFC_KMAX,
    GFC_NOALLOC_MAX_GALAXIES,
    GFC_RAMP_LINEAR,
    GFC_SHIFT_LANCZOS3,
    GfcError,
    LIB_PATH,
    lib,
)
from .api import (  # noqa: F401
    Context,
    Mixture,
    Psf,
    SersicFamily,
    gfc_backward_workspace_bytes,
    gfc_render_stamps,
    gfc_render_stamps_backward,
    gfc_render_stamps_backward_noalloc,
    gfc_render_stamps_composite,
    gfc_render_stamps_sersic,
)
from .autograd import RenderStamps, render  # noqa: F401,E402
