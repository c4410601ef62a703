// Internal host-side definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gfc.h"
#include "gfc_device.hpp"
#include "gfc_error.hpp"

struct gfc_ctx {
  int device = 0;
  unsigned long long* d_invalid = nullptr;  // device counter of invalid galaxies
  std::atomic<int> n_objects{0};            // PSFs, mixtures and servers alive
};

namespace gfc {
// Cached PSF spectrum for one stamp size W: columns 0..W/2-1 in the order
// the render kernels' lanes read them, then the Nyquist column.
struct PsfSpectrum {
  int W = 0;
  float2* main_cols = nullptr;  // [W/2][W] (one allocation with nyq_col)
  float2* nyq_col = nullptr;    // [W]
  int64_t stride = 0;           // float2 from one eigen-PSF component's spectrum to the next
};
}  // namespace gfc

struct gfc_psf {
  gfc_ctx* ctx = nullptr;
  uint64_t uid = 0;  // unique in the process (a later PSF at the same address has another)
  int Sy = 0, Sx = 0;
  double* d_pix = nullptr;  // device, float64 [J or 1][Sy][Sx]
  double gauss[6] = {0, 0, 0, 0, 0, 0};
  // Spatially varying (eigen-)PSF: J > 0 components with polynomial weights.
  int J = 0;
  int degree = 0;
  double norm[4] = {0, 1, 0, 1};  // x_off, x_scale, y_off, y_scale
  float* d_eig = nullptr;         // device: coefficients [J][T], then raw moments [J][6]
  std::mutex mu;
  std::map<int, gfc::PsfSpectrum> cache;
};

struct gfc_mix {
  gfc_ctx* ctx = nullptr;
  int n_tables = 0;
  int kmax = 0;
  float* d_amp = nullptr;  // [n_tables][GFC_KMAX]
  float* d_var = nullptr;
  int32_t* d_K = nullptr;
  std::vector<int32_t> K;  // host copy of the component counts
};

namespace gfc {

gfc_status hip_fail(hipError_t e, const char* what);  // fail() with the HIP error's text
bool stamp_size_ok(int W);

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;

 private:
  int prev_ = -1;
};

gfc_status psf_cache(gfc_psf* psf, int W, hipStream_t stream, const PsfSpectrum** out);
// Next process-unique PSF id.
uint64_t next_psf_uid();
// The cached spectrum for W, or nullptr when it has not been filled (never fills).
const PsfSpectrum* psf_cache_find(gfc_psf* psf, int W);
// Takes the device address of the allocation-free adjoint's scratch array on
// `device` (current); once per device, from gfc_ctx_create.
gfc_status noalloc_scratch_setup(int device);
gfc_status fill_render_args(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, const gfc_galaxies* gal,
                            int64_t n, int W, unsigned flags, RenderArgs* a);
// Points the render arguments at a cached spectrum.
void attach_spectrum(RenderArgs* a, const PsfSpectrum* spec);
// Launches the forward kernels for stamp size W (arguments already validated).
gfc_status render_launch(const RenderArgs& a, int W, hipStream_t stream);

}  // namespace gfc
