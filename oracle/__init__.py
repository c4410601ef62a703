"""FP64 CPU oracle for the hybrid Fourier-real mixture-of-Gaussians
galaxy-PSF convolution (Lang 2020, arXiv:2012.15797, Section 2).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product (the HIP
library and its Python binding) never imports, links or executes it, and it
shares no code, table or constant generator with the product.

It is deliberately plain and slow: naive separable DFT matrices, direct
evaluation of every Gaussian, float64/complex128 throughout.

Parity status of each function is recorded in its docstring.  Every function
is pinned by a test in tests/test_oracle_*.py against something other than
itself (closed forms, invariants, library routines, brute force, finite
differences); the one exception is the real-world accuracy of a mixture
approximation to a Sersic profile, which the paper's missing tables would be
needed for and which is out of scope.
"""

from .render import (  # noqa: F401
    FORCE_FOURIER,
    FORCE_REAL,
    RAMP_LINEAR,
    fold_psf,
    psf_spectrum,
    psf_gauss_moments,
    covariances,
    routing_weights,
    axis_frequencies,
    galaxy_spectrum,
    inverse_dft2,
    real_space_image,
    render_stamp,
    render_batch,
)
from .grad import render_stamp_jacobian, loss_gradient, fd_gradient  # noqa: F401
