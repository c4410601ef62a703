// Host side of the C ABI declared in include/gfc.h: contexts, PSF-FT caches,
// mixture tables, argument validation and kernel launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gfc.h"
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"
#include "gfc_trace.hpp"

using gfc::RenderArgs;

namespace gfc {

gfc_status hip_fail(hipError_t e, const char* what) {
  return fail(GFC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
  if (prev_ != dev) hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
  if (prev_ >= 0) hipSetDevice(prev_);
}

bool stamp_size_ok(int W) { return W == 16 || W == 32 || W == 64 || W == 128 || W == 256; }

// Fills (once) and returns the PSF-FT cache entry for stamp size W.
gfc_status psf_cache(gfc_psf* psf, int W, hipStream_t stream, const PsfSpectrum** out) {
  std::lock_guard<std::mutex> lock(psf->mu);
  auto it = psf->cache.find(W);
  if (it != psf->cache.end()) {
    *out = &it->second;
    return GFC_OK;
  }
  TraceScope trace("gfc psf cache fill");
  const auto t0 = std::chrono::steady_clock::now();
  PsfSpectrum spec;
  const size_t main_n = (size_t)(W / 2) * W, nyq_n = (size_t)W;
  const int ncomp = psf->J > 0 ? psf->J : 1;
  spec.stride = (int64_t)(main_n + nyq_n);
  hipError_t e = hipMalloc(&spec.main_cols, (size_t)ncomp * (main_n + nyq_n) * sizeof(float2));
  if (e != hipSuccess) return fail(GFC_ENOMEM, "PSF cache allocation failed");
  spec.nyq_col = spec.main_cols + main_n;
  double2* tmp = nullptr;
  e = hipMalloc(&tmp, (size_t)psf->Sy * (W / 2 + 1) * sizeof(double2));
  if (e != hipSuccess) {
    hipFree(spec.main_cols);
    return fail(GFC_ENOMEM, "PSF cache scratch allocation failed");
  }
  // One transform per component (one for a constant PSF); the same stream
  // orders the reuse of tmp.
  for (int j = 0; j < ncomp && e == hipSuccess; ++j)
    e = launch_psf_spectrum(psf->d_pix + (size_t)j * psf->Sy * psf->Sx, psf->Sy, psf->Sx, W, tmp,
                            spec.main_cols + j * spec.stride, spec.nyq_col + j * spec.stride, nullptr,
                            stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  hipFree(tmp);
  if (e != hipSuccess) {
    hipFree(spec.main_cols);
    return hip_fail(e, "PSF spectrum");
  }
  spec.W = W;
  auto ins = psf->cache.emplace(W, spec);
  *out = &ins.first->second;
  if (log_enabled())
    log_event("psf_cache_fill", "\"psf\": " + std::to_string(psf->uid) + ", \"W\": " + std::to_string(W) +
                                    ", \"components\": " + std::to_string(ncomp) + ", \"ms\": " +
                                    std::to_string(std::chrono::duration<double, std::milli>(
                                                       std::chrono::steady_clock::now() - t0).count()));
  return GFC_OK;
}

uint64_t next_psf_uid() {
  static std::atomic<uint64_t> next{1};
  return next.fetch_add(1);
}

const PsfSpectrum* psf_cache_find(gfc_psf* psf, int W) {
  std::lock_guard<std::mutex> lock(psf->mu);
  const auto it = psf->cache.find(W);
  return it == psf->cache.end() ? nullptr : &it->second;
}

gfc_status fill_render_args(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, const gfc_galaxies* gal,
                            int64_t n, int W, unsigned flags, RenderArgs* a) {
  if (!ctx || !psf || !mix || !gal) return fail(GFC_EINVAL, "null handle or galaxy block");
  if (psf->ctx != ctx || mix->ctx != ctx) return fail(GFC_EINVAL, "handle belongs to another context");
  if (!stamp_size_ok(W)) return fail(GFC_EINVAL, "stamp size must be 16, 32, 64, 128 or 256");
  if (n < 0) return fail(GFC_EINVAL, "negative galaxy count");
  if ((flags & ~31u) != 0) return fail(GFC_EINVAL, "unknown flag bits");
  if ((flags & GFC_SHIFT_LANCZOS3) && (flags & GFC_ACCUMULATE))
    return fail(GFC_EINVAL, "GFC_ACCUMULATE cannot be combined with GFC_SHIFT_LANCZOS3");
  if ((flags & GFC_FORCE_FOURIER) && (flags & GFC_FORCE_REAL))
    return fail(GFC_EINVAL, "GFC_FORCE_FOURIER and GFC_FORCE_REAL are exclusive");
  if (n > 0 && (!gal->x || !gal->y || !gal->flux || !gal->r_e || !gal->e1 || !gal->e2))
    return fail(GFC_EINVAL, "null galaxy parameter array");
  std::memset(a, 0, sizeof(*a));
  a->x = gal->x;
  a->y = gal->y;
  a->flux = gal->flux;
  a->r_e = gal->r_e;
  a->e1 = gal->e1;
  a->e2 = gal->e2;
  a->mix_id = gal->mix_id;
  a->amp = gal->mix_amp ? gal->mix_amp : mix->d_amp;  // a per-call amplitude table leaves the mixture as it is
  a->var = mix->d_var;
  a->K = mix->d_K;
  a->n_tables = mix->n_tables;
  a->kmax = mix->kmax;
  if (gal->cd) {
    const double t = gal->cd[0], u = gal->cd[1], v = gal->cd[2], w = gal->cd[3];
    const double det = t * w - u * v;
    if (!(std::isfinite(det) && det != 0.0)) return fail(GFC_EINVAL, "CD matrix is singular");
    a->cdinv[0] = (float)(w / det);
    a->cdinv[1] = (float)(-u / det);
    a->cdinv[2] = (float)(-v / det);
    a->cdinv[3] = (float)(t / det);
  } else {
    a->cdinv[0] = 1.f;
    a->cdinv[3] = 1.f;
  }
  for (int i = 0; i < 6; ++i) a->pg[i] = (float)psf->gauss[i];
  if (psf->J > 0) {
    if (n > 0 && (!gal->psf_x || !gal->psf_y))
      return fail(GFC_EINVAL, "a spatially varying PSF needs psf_x and psf_y for every galaxy");
    const int T = (psf->degree + 1) * (psf->degree + 2) / 2;
    a->eig_J = psf->J;
    a->eig_degree = psf->degree;
    a->eig_coef = psf->d_eig;
    a->eig_mom = psf->d_eig + (size_t)psf->J * T;
    a->eig_norm[0] = (float)psf->norm[0];
    a->eig_norm[1] = (float)(1.0 / psf->norm[1]);
    a->eig_norm[2] = (float)psf->norm[2];
    a->eig_norm[3] = (float)(1.0 / psf->norm[3]);
    a->psf_px = gal->psf_x;
    a->psf_py = gal->psf_y;
  }
  a->n = n;
  a->flags = flags;
  a->invalid = ctx->d_invalid;
  return GFC_OK;
}

void attach_spectrum(RenderArgs* a, const PsfSpectrum* spec) {
  a->psf_main = spec->main_cols;
  a->psf_nyq = spec->nyq_col;
  a->eig_stride = spec->stride;
}

}  // namespace gfc

using namespace gfc;

extern "C" {

int gfc_stamp_size_supported(int W) { return stamp_size_ok(W) ? 1 : 0; }

gfc_status gfc_ctx_create(int hip_device, gfc_ctx** out) {
  if (!out) return fail(GFC_EINVAL, "null output pointer");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= count) return fail(GFC_EINVAL, "no such HIP device");
  DeviceGuard guard(hip_device);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GFC_EUNSUPPORTED, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
  const gfc_status st = noalloc_scratch_setup(hip_device);
  if (st != GFC_OK) return st;
  auto* ctx = new (std::nothrow) gfc_ctx();
  if (!ctx) return fail(GFC_ENOMEM, "context allocation failed");
  ctx->device = hip_device;
  e = hipMalloc(&ctx->d_invalid, sizeof(unsigned long long));
  if (e != hipSuccess) {
    delete ctx;
    return fail(GFC_ENOMEM, "invalid-counter allocation failed");
  }
  // Stream-ordered scratch (the W = 256 adjoint's slab, the adjoint
  // workspace, per-galaxy mixture tables, serving fallbacks) comes from the
  // device's default memory pool; keep freed blocks
  // cached in it instead of returning them to the HIP runtime at every
  // synchronisation, so repeated calls do not pay for fresh allocations.
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, hip_device) == hipSuccess && pool) {
    uint64_t keep = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  e = hipMemset(ctx->d_invalid, 0, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hipFree(ctx->d_invalid);
    delete ctx;
    return hip_fail(e, "context init");
  }
  *out = ctx;
  return GFC_OK;
}

gfc_status gfc_ctx_destroy(gfc_ctx* ctx) {
  if (!ctx) return fail(GFC_EINVAL, "null context");
  if (ctx->n_objects.load() != 0) return fail(GFC_EBUSY, "context still owns PSFs, mixtures or servers");
  DeviceGuard guard(ctx->device);
  hipDeviceSynchronize();
  hipFree(ctx->d_invalid);
  delete ctx;
  return GFC_OK;
}

gfc_status gfc_ctx_invalid_count(gfc_ctx* ctx, uint64_t* n_invalid) {
  if (!ctx || !n_invalid) return fail(GFC_EINVAL, "null argument");
  DeviceGuard guard(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  unsigned long long v = 0;
  e = hipMemcpy(&v, ctx->d_invalid, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read invalid counter");
  *n_invalid = v;
  return GFC_OK;
}

static gfc_status psf_create_impl(gfc_ctx* ctx, const double* pix, int Sy, int Sx, const double* gauss,
                                  gfc_psf** out) {
  if (!ctx || !pix || !out) return fail(GFC_EINVAL, "null argument");
  *out = nullptr;
  if (Sy < 2 || Sx < 2 || Sy > 1024 || Sx > 1024 || (Sy & 1) || (Sx & 1))
    return fail(GFC_EINVAL, "PSF sides must be even, 2..1024");
  const size_t npix = (size_t)Sy * Sx;
  double sum = 0.0;
  for (size_t i = 0; i < npix; ++i) {
    if (!std::isfinite(pix[i])) return fail(GFC_EINVAL, "non-finite PSF pixel");
    sum += pix[i];
  }
  double g[6];
  if (gauss) {
    for (int i = 0; i < 6; ++i) {
      if (!std::isfinite(gauss[i])) return fail(GFC_EINVAL, "non-finite PSF Gaussian");
      g[i] = gauss[i];
    }
  } else {
    // Moments about the centre pixel (S_y/2, S_x/2), amplitude = pixel sum.
    if (!(sum > 0.0)) return fail(GFC_EINVAL, "PSF pixel sum must be positive for moment matching");
    double mx = 0, my = 0;
    for (int r = 0; r < Sy; ++r)
      for (int c = 0; c < Sx; ++c) {
        const double p = pix[(size_t)r * Sx + c];
        mx += p * (c - Sx / 2);
        my += p * (r - Sy / 2);
      }
    mx /= sum;
    my /= sum;
    double cxx = 0, cxy = 0, cyy = 0;
    for (int r = 0; r < Sy; ++r)
      for (int c = 0; c < Sx; ++c) {
        const double p = pix[(size_t)r * Sx + c];
        const double dx = (c - Sx / 2) - mx, dy = (r - Sy / 2) - my;
        cxx += p * dx * dx;
        cxy += p * dx * dy;
        cyy += p * dy * dy;
      }
    g[0] = mx;
    g[1] = my;
    g[2] = cxx / sum;
    g[3] = cxy / sum;
    g[4] = cyy / sum;
    g[5] = sum;
  }
  if (g[2] < 0 || g[4] < 0 || g[2] * g[4] - g[3] * g[3] < 0)
    return fail(GFC_EINVAL, "PSF Gaussian covariance is not positive semi-definite");
  DeviceGuard guard(ctx->device);
  auto* psf = new (std::nothrow) gfc_psf();
  if (!psf) return fail(GFC_ENOMEM, "PSF allocation failed");
  psf->ctx = ctx;
  psf->uid = next_psf_uid();
  psf->Sy = Sy;
  psf->Sx = Sx;
  std::memcpy(psf->gauss, g, sizeof(g));
  hipError_t e = hipMalloc(&psf->d_pix, npix * sizeof(double));
  if (e != hipSuccess) {
    delete psf;
    return fail(GFC_ENOMEM, "PSF pixel allocation failed");
  }
  e = hipMemcpy(psf->d_pix, pix, npix * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(psf->d_pix);
    delete psf;
    return hip_fail(e, "PSF upload");
  }
  ctx->n_objects++;
  *out = psf;
  return GFC_OK;
}

gfc_status gfc_psf_create_f64(gfc_ctx* ctx, const double* pix, int Sy, int Sx, const double* gauss,
                              gfc_psf** out) {
  return psf_create_impl(ctx, pix, Sy, Sx, gauss, out);
}

gfc_status gfc_psf_create(gfc_ctx* ctx, const float* pix, int Sy, int Sx, const double* gauss,
                          gfc_psf** out) {
  if (!pix || Sy <= 0 || Sx <= 0 || Sy > 1024 || Sx > 1024)
    return fail(GFC_EINVAL, "bad PSF pixel array");
  std::vector<double> d((size_t)Sy * Sx);
  for (size_t i = 0; i < d.size(); ++i) d[i] = pix[i];
  return psf_create_impl(ctx, d.data(), Sy, Sx, gauss, out);
}

gfc_status gfc_psf_create_eigen(gfc_ctx* ctx, const float* comps, int J, int Sy, int Sx, int degree,
                                const double* coef, const double* norm, gfc_psf** out) {
  if (!ctx || !comps || !coef || !norm || !out) return fail(GFC_EINVAL, "null argument");
  *out = nullptr;
  if (J < 1 || J > kEigMax) return fail(GFC_EINVAL, "eigen-PSF needs 1..16 components");
  if (degree < 0 || degree > kEigDegMax) return fail(GFC_EINVAL, "eigen-PSF polynomial degree must be 0..3");
  if (Sy < 2 || Sx < 2 || Sy > 1024 || Sx > 1024 || (Sy & 1) || (Sx & 1))
    return fail(GFC_EINVAL, "PSF sides must be even, 2..1024");
  if (!(std::isfinite(norm[0]) && std::isfinite(norm[2]) && std::isfinite(norm[1]) && std::isfinite(norm[3]) &&
        norm[1] != 0.0 && norm[3] != 0.0))
    return fail(GFC_EINVAL, "eigen-PSF normalisation must be finite with non-zero scales");
  const int T = (degree + 1) * (degree + 2) / 2;
  const size_t npix = (size_t)Sy * Sx;
  std::vector<double> pix((size_t)J * npix);
  // device block: coefficients [J][T] then raw moments about the centre pixel [J][6]
  std::vector<float> eig((size_t)J * T + (size_t)J * 6);
  for (int j = 0; j < J; ++j) {
    for (int t = 0; t < T; ++t) {
      const double c = coef[(size_t)j * T + t];
      if (!std::isfinite(c)) return fail(GFC_EINVAL, "non-finite eigen-PSF coefficient");
      eig[(size_t)j * T + t] = (float)c;
    }
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < Sy; ++r)
      for (int c = 0; c < Sx; ++c) {
        const double v = comps[(size_t)j * npix + (size_t)r * Sx + c];
        if (!std::isfinite(v)) return fail(GFC_EINVAL, "non-finite eigen-PSF pixel");
        pix[(size_t)j * npix + (size_t)r * Sx + c] = v;
        const double x = c - Sx / 2, y = r - Sy / 2;
        m[0] += v;
        m[1] += v * x;
        m[2] += v * y;
        m[3] += v * x * x;
        m[4] += v * x * y;
        m[5] += v * y * y;
      }
    for (int i = 0; i < 6; ++i) eig[(size_t)J * T + (size_t)j * 6 + i] = (float)m[i];
  }
  DeviceGuard guard(ctx->device);
  auto* psf = new (std::nothrow) gfc_psf();
  if (!psf) return fail(GFC_ENOMEM, "PSF allocation failed");
  psf->ctx = ctx;
  psf->uid = next_psf_uid();
  psf->Sy = Sy;
  psf->Sx = Sx;
  psf->J = J;
  psf->degree = degree;
  std::memcpy(psf->norm, norm, sizeof(psf->norm));
  hipError_t e = hipMalloc(&psf->d_pix, pix.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&psf->d_eig, eig.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(psf->d_pix, pix.data(), pix.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(psf->d_eig, eig.data(), eig.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(psf->d_pix);
    hipFree(psf->d_eig);
    delete psf;
    return hip_fail(e, "eigen-PSF upload");
  }
  ctx->n_objects++;
  *out = psf;
  return GFC_OK;
}

gfc_status gfc_psf_gauss(const gfc_psf* psf, double* gauss_out) {
  if (!psf || !gauss_out) return fail(GFC_EINVAL, "null argument");
  if (psf->J > 0) return fail(GFC_EUNSUPPORTED, "the Gaussian of a spatially varying PSF depends on position");
  std::memcpy(gauss_out, psf->gauss, sizeof(psf->gauss));
  return GFC_OK;
}

gfc_status gfc_psf_prepare(gfc_psf* psf, int W, void* hip_stream) {
  if (!psf) return fail(GFC_EINVAL, "null PSF");
  if (!stamp_size_ok(W)) return fail(GFC_EINVAL, "unsupported stamp size");
  DeviceGuard guard(psf->ctx->device);
  const PsfSpectrum* spec = nullptr;
  return psf_cache(psf, W, (hipStream_t)hip_stream, &spec);
}

gfc_status gfc_psf_spectrum(gfc_psf* psf, int W, float* spec_out, void* hip_stream) {
  if (!psf || !spec_out) return fail(GFC_EINVAL, "null argument");
  if (!stamp_size_ok(W)) return fail(GFC_EINVAL, "unsupported stamp size");
  DeviceGuard guard(psf->ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const PsfSpectrum* spec = nullptr;
  gfc_status st = psf_cache(psf, W, s, &spec);
  if (st != GFC_OK) return st;
  // Recompute into the natural layout (a debugging and test view of the cache).
  double2* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, (size_t)psf->Sy * (W / 2 + 1) * sizeof(double2));
  if (e != hipSuccess) return fail(GFC_ENOMEM, "scratch allocation failed");
  float2 *m = nullptr;
  e = hipMalloc(&m, ((size_t)(W / 2) * W + W) * sizeof(float2));
  if (e != hipSuccess) {
    hipFree(tmp);
    return fail(GFC_ENOMEM, "scratch allocation failed");
  }
  const int ncomp = psf->J > 0 ? psf->J : 1;
  for (int j = 0; j < ncomp && e == hipSuccess; ++j)
    e = launch_psf_spectrum(psf->d_pix + (size_t)j * psf->Sy * psf->Sx, psf->Sy, psf->Sx, W, tmp, m,
                            m + (size_t)(W / 2) * W,
                            reinterpret_cast<float2*>(spec_out) + (size_t)j * W * (W / 2 + 1), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(tmp);
  hipFree(m);
  if (e != hipSuccess) return hip_fail(e, "PSF spectrum");
  return GFC_OK;
}

gfc_status gfc_psf_destroy(gfc_psf* psf) {
  if (!psf) return fail(GFC_EINVAL, "null PSF");
  DeviceGuard guard(psf->ctx->device);
  hipDeviceSynchronize();
  for (auto& kv : psf->cache) hipFree(kv.second.main_cols);
  hipFree(psf->d_pix);
  hipFree(psf->d_eig);
  psf->ctx->n_objects--;
  delete psf;
  return GFC_OK;
}

gfc_status gfc_mix_create(gfc_ctx* ctx, int n_tables, const int* K, const float* amp, const float* var,
                          gfc_mix** out) {
  if (!ctx || !K || !amp || !var || !out) return fail(GFC_EINVAL, "null argument");
  *out = nullptr;
  if (n_tables < 1 || n_tables > (1 << 20)) return fail(GFC_EINVAL, "n_tables out of range");
  std::vector<float> a((size_t)n_tables * GFC_KMAX, 0.f), v((size_t)n_tables * GFC_KMAX, 1.f);
  int kmax = 0;
  for (int t = 0; t < n_tables; ++t) {
    if (K[t] < 1 || K[t] > GFC_KMAX) return fail(GFC_EINVAL, "mixture size must be 1..16");
    kmax = std::max(kmax, K[t]);
    for (int k = 0; k < K[t]; ++k) {
      const float ak = amp[(size_t)t * GFC_KMAX + k], vk = var[(size_t)t * GFC_KMAX + k];
      if (!std::isfinite(ak) || !std::isfinite(vk) || !(vk > 0.f))
        return fail(GFC_EINVAL, "mixture amplitudes must be finite and variances positive");
      a[(size_t)t * GFC_KMAX + k] = ak;
      v[(size_t)t * GFC_KMAX + k] = vk;
    }
  }
  DeviceGuard guard(ctx->device);
  auto* mix = new (std::nothrow) gfc_mix();
  if (!mix) return fail(GFC_ENOMEM, "mixture allocation failed");
  mix->ctx = ctx;
  mix->n_tables = n_tables;
  mix->kmax = kmax;
  mix->K.assign(K, K + n_tables);
  const size_t nb = (size_t)n_tables * GFC_KMAX * sizeof(float);
  hipError_t e = hipMalloc(&mix->d_amp, nb);
  if (e == hipSuccess) e = hipMalloc(&mix->d_var, nb);
  if (e == hipSuccess) e = hipMalloc(&mix->d_K, n_tables * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(mix->d_amp, a.data(), nb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mix->d_var, v.data(), nb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mix->d_K, K, n_tables * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(mix->d_amp);
    hipFree(mix->d_var);
    hipFree(mix->d_K);
    delete mix;
    return hip_fail(e, "mixture upload");
  }
  ctx->n_objects++;
  *out = mix;
  return GFC_OK;
}

gfc_status gfc_mix_device_tables(gfc_mix* mix, float** amp_dev, float** var_dev) {
  if (!mix) return fail(GFC_EINVAL, "null mixture");
  if (amp_dev) *amp_dev = mix->d_amp;
  if (var_dev) *var_dev = mix->d_var;
  return GFC_OK;
}

gfc_status gfc_mix_set_amp(gfc_mix* mix, const float* amp_dev, void* hip_stream) {
  if (!mix || !amp_dev) return fail(GFC_EINVAL, "null argument");
  DeviceGuard guard(mix->ctx->device);
  hipError_t e = hipMemcpyAsync(mix->d_amp, amp_dev, (size_t)mix->n_tables * GFC_KMAX * sizeof(float),
                                hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "amplitude copy");
  return GFC_OK;
}

gfc_status gfc_mix_destroy(gfc_mix* mix) {
  if (!mix) return fail(GFC_EINVAL, "null mixture");
  DeviceGuard guard(mix->ctx->device);
  hipDeviceSynchronize();
  hipFree(mix->d_amp);
  hipFree(mix->d_var);
  hipFree(mix->d_K);
  mix->ctx->n_objects--;
  delete mix;
  return GFC_OK;
}

gfc_status gfc_render_stamps(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, const gfc_galaxies* gal,
                             int64_t n, int W, unsigned flags, float* out, void* hip_stream) {
  TraceScope trace("gfc render");
  RenderArgs a;
  gfc_status st = fill_render_args(ctx, psf, mix, gal, n, W, flags, &a);
  if (st != GFC_OK) return st;
  if (n == 0) return GFC_OK;
  if (!out) return fail(GFC_EINVAL, "null output");
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const PsfSpectrum* spec = nullptr;
  st = psf_cache(psf, W, s, &spec);
  if (st != GFC_OK) return st;
  attach_spectrum(&a, spec);
  a.out = out;
  if (log_enabled())
    log_event("render", "\"n\": " + std::to_string(n) + ", \"W\": " + std::to_string(W) + ", \"flags\": " +
                            std::to_string(flags));
  return render_launch(a, W, s);
}

}  // extern "C"
