// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gfc_device.hpp"

namespace gfc {

// Forward render, W in {16, 32, 64, 128}.
template <int W>
hipError_t launch_render_small(const RenderArgs& args, hipStream_t stream);

// Forward render, W = 256 (device scratch allocated stream-ordered per call).
hipError_t launch_render_w256(const RenderArgs& args, hipStream_t stream);

// Adjoint, W = 256: per-stamp parameter gradients and amplitude partials
// (device scratch allocated stream-ordered per call).
hipError_t launch_bwd_w256(const RenderArgs& args, const float* gout, float* grad_params, float* amp_part,
                           hipStream_t stream);

// Lanczos-3 shift of the finished stamps a.out by the fractional parts of
// a.x, a.y (Section 2, step 8 alternative), in place; W = 128 or 256 (the
// smaller sizes shift inside the render kernel).
hipError_t launch_lanczos_shift(const RenderArgs& a, int W, hipStream_t stream);

// PSF spectrum (Section 2, steps 1-2): separable float64 DFT of the S_y x S_x
// PSF with its centre pixel at frequency-grid index 0.  Writes the
// lane-permuted main columns, the Nyquist column and optionally the natural
// [W][W/2+1] layout.  tmp: device, S_y * (W/2+1) double2.
hipError_t launch_psf_spectrum(const double* pix, int Sy, int Sx, int W, double2* tmp,
                               float2* main_cols, float2* nyq_col, float2* natural,
                               hipStream_t stream);

}  // namespace gfc
