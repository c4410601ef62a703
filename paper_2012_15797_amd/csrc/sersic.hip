// General-Sérsic and composite (bulge + disk) galaxies (Lang 2020: Section 1
// on the profile family and its bulge-disk combinations; the closing
// discussion on interpolating mixture parameters between Sérsic indices).
//
// Both reduce to the ordinary render with one mixture per galaxy.  A small
// pre-pass writes each galaxy's mixture (amplitudes, variances, K) and a
// table index into stream-ordered scratch; the forward kernels then run
// unchanged with one table per galaxy.  An invalid profile parameter gives
// the galaxy an out-of-range table index, which the render turns into a NaN
// stamp and counts.
#include <cmath>
#include <cstring>
#include <vector>

#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

struct gfc_sersic {
  gfc_ctx* ctx = nullptr;
  int S = 0, K = 0;
  float* d_grid = nullptr;  // [S] indices, then amp [S][K], then var [S][K]
};

namespace gfc {
namespace {

constexpr int kPre = 256;

struct PerGalaxyTables {
  float* amp;    // [n][kKmax]
  float* var;    // [n][kKmax]
  int32_t* K;    // [n]
  int32_t* id;   // [n]: the galaxy's own index, or -1 if its profile is invalid
};

// The per-galaxy tables are written one thread per (galaxy, component)
// element, so a wavefront's stores are contiguous ([n][kKmax] row-major);
// the galaxy's scalars are read by its kKmax threads from one cache line.

// Piecewise-linear interpolation in n of each component's amplitude and
// variance between the two grid indices around n.
__global__ void __launch_bounds__(kPre) sersic_tables_kernel(const float* __restrict__ sersic_n, int S,
                                                             const float* __restrict__ grid, int K, int64_t n,
                                                             PerGalaxyTables t) {
  // the grid indices staged in LDS once per block (S <= 256 = kPre), so the
  // search below does not wait on one scalar load per index
  __shared__ float s_grid[kPre];
  if ((int)threadIdx.x < S) s_grid[threadIdx.x] = grid[threadIdx.x];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * kPre + threadIdx.x;
  if (e >= n * kKmax) return;
  const int64_t g = e / kKmax;
  const int k = (int)(e % kKmax);
  const float* amp = grid + S;
  const float* var = amp + S * K;
  const float nn = sersic_n[g];
  const bool ok = __builtin_isfinite(nn) && nn >= s_grid[0] && nn <= s_grid[S - 1];
  int s = 0;
  for (int i = 1; i < S - 1; ++i)
    if (s_grid[i] <= nn) s = i;
  const float t1 = ok ? (nn - s_grid[s]) / (s_grid[s + 1] - s_grid[s]) : 0.f, t0 = 1.f - t1;
  float a = 0.f, v = 1.f;
  if (k < K) {
    a = fmaf(t0, amp[s * K + k], t1 * amp[(s + 1) * K + k]);
    v = fmaf(t0, var[s * K + k], t1 * var[(s + 1) * K + k]);
  }
  t.amp[e] = a;
  t.var[e] = v;
  if (k == 0) {
    t.K[g] = K;
    t.id[g] = ok ? (int32_t)g : -1;
  }
}

// One-ellipticity composite: disk components with amplitudes (1 - f) A_d,
// bulge components with amplitudes f A_b and variances rho^2 v_b.
__global__ void __launch_bounds__(kPre) composite_tables_kernel(
    const float* __restrict__ mamp, const float* __restrict__ mvar, int disk, int Kd, int bulge, int Kb,
    const float* __restrict__ frac, const float* __restrict__ rho, int64_t n, PerGalaxyTables t) {
  const int64_t e = (int64_t)blockIdx.x * kPre + threadIdx.x;
  if (e >= n * kKmax) return;
  const int64_t g = e / kKmax;
  const int k = (int)(e % kKmax);
  const float f = frac[g], r = rho[g];
  const bool ok = f >= 0.f && f <= 1.f && r > 0.f && __builtin_isfinite(r);
  float a = 0.f, v = 1.f;
  if (k < Kd) {
    a = (1.f - f) * mamp[disk * kKmax + k];
    v = mvar[disk * kKmax + k];
  } else if (k < Kd + Kb) {
    a = f * mamp[bulge * kKmax + (k - Kd)];
    v = (r * r) * mvar[bulge * kKmax + (k - Kd)];
  }
  t.amp[e] = a;
  t.var[e] = v;
  if (k == 0) {
    t.K[g] = Kd + Kb;
    t.id[g] = ok ? (int32_t)g : -1;
  }
}

// Blocks for one thread per table element.
inline unsigned table_blocks(int64_t n) { return (unsigned)((n * kKmax + kPre - 1) / kPre); }

// Scratch for the per-galaxy tables, stream-ordered.
gfc_status alloc_tables(int64_t n, hipStream_t s, void** block, PerGalaxyTables* t) {
  const size_t fbytes = (size_t)n * kKmax * sizeof(float);
  const size_t ibytes = (size_t)n * sizeof(int32_t);
  if (hipMallocAsync(block, 2 * fbytes + 2 * ibytes, s) != hipSuccess)
    return fail(GFC_ENOMEM, "per-galaxy mixture scratch allocation failed");
  char* b = static_cast<char*>(*block);
  t->amp = reinterpret_cast<float*>(b);
  t->var = reinterpret_cast<float*>(b + fbytes);
  t->K = reinterpret_cast<int32_t*>(b + 2 * fbytes);
  t->id = reinterpret_cast<int32_t*>(b + 2 * fbytes + ibytes);
  return GFC_OK;
}

// Common tail: validate, fill the cache, launch the pre-pass and the render
// with one table per galaxy.
template <typename PrePass>
gfc_status render_per_galaxy(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix_like, int kmax,
                             const gfc_galaxies* gal, int64_t n, int W, unsigned flags, float* out,
                             hipStream_t s, PrePass prepass) {
  if (n > (int64_t)INT32_MAX) return fail(GFC_EINVAL, "at most 2^31 - 1 galaxies per call with per-galaxy mixtures");
  RenderArgs a;
  gfc_status st = fill_render_args(ctx, psf, mix_like, gal, n, W, flags, &a);
  if (st != GFC_OK) return st;
  if (n == 0) return GFC_OK;
  if (!out) return fail(GFC_EINVAL, "null output");
  DeviceGuard guard(ctx->device);
  const PsfSpectrum* spec = nullptr;
  st = psf_cache(psf, W, s, &spec);
  if (st != GFC_OK) return st;
  void* block = nullptr;
  PerGalaxyTables t;
  st = alloc_tables(n, s, &block, &t);
  if (st != GFC_OK) return st;
  hipError_t e = prepass(t);
  if (e == hipSuccess) {
    attach_spectrum(&a, spec);
    a.amp = t.amp;
    a.var = t.var;
    a.K = t.K;
    a.mix_id = t.id;
    a.n_tables = (int)n;
    a.kmax = kmax;
    a.out = out;
    st = render_launch(a, W, s);
  } else {
    st = hip_fail(e, "per-galaxy mixture pre-pass");
  }
  hipError_t e2 = hipFreeAsync(block, s);
  if (st == GFC_OK && e2 != hipSuccess) st = hip_fail(e2, "per-galaxy mixture scratch release");
  return st;
}

}  // namespace
}  // namespace gfc

using namespace gfc;

extern "C" {

gfc_status gfc_sersic_create(gfc_ctx* ctx, int S, const float* n_grid, int K, const float* amp, const float* var,
                             gfc_sersic** out) {
  if (!ctx || !n_grid || !amp || !var || !out) return fail(GFC_EINVAL, "null argument");
  *out = nullptr;
  if (S < 2 || S > 256) return fail(GFC_EINVAL, "a Sersic family needs 2..256 grid indices");
  if (K < 1 || K > kKmax) return fail(GFC_EINVAL, "a Sersic family needs 1..16 components");
  for (int i = 0; i < S; ++i) {
    if (!std::isfinite(n_grid[i]) || (i > 0 && !(n_grid[i] > n_grid[i - 1])))
      return fail(GFC_EINVAL, "Sersic grid indices must be finite and strictly increasing");
    for (int k = 0; k < K; ++k) {
      if (!std::isfinite(amp[i * K + k])) return fail(GFC_EINVAL, "non-finite Sersic amplitude");
      if (!(var[i * K + k] > 0.f) || !std::isfinite(var[i * K + k]))
        return fail(GFC_EINVAL, "Sersic variances must be positive and finite");
    }
  }
  DeviceGuard guard(ctx->device);
  auto* f = new (std::nothrow) gfc_sersic();
  if (!f) return fail(GFC_ENOMEM, "allocation failed");
  f->ctx = ctx;
  f->S = S;
  f->K = K;
  std::vector<float> h((size_t)S + 2 * (size_t)S * K);
  std::memcpy(h.data(), n_grid, S * sizeof(float));
  std::memcpy(h.data() + S, amp, (size_t)S * K * sizeof(float));
  std::memcpy(h.data() + S + (size_t)S * K, var, (size_t)S * K * sizeof(float));
  hipError_t e = hipMalloc(&f->d_grid, h.size() * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(f->d_grid, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(f->d_grid);
    delete f;
    return hip_fail(e, "Sersic family upload");
  }
  ctx->n_objects++;
  *out = f;
  return GFC_OK;
}

gfc_status gfc_sersic_destroy(gfc_sersic* f) {
  if (!f) return fail(GFC_EINVAL, "null Sersic family");
  DeviceGuard guard(f->ctx->device);
  hipDeviceSynchronize();
  hipFree(f->d_grid);
  f->ctx->n_objects--;
  delete f;
  return GFC_OK;
}

gfc_status gfc_render_stamps_sersic(gfc_ctx* ctx, gfc_psf* psf, const gfc_sersic* fam, const gfc_galaxies* gal,
                                    const float* sersic_n, int64_t n, int W, unsigned flags, float* out,
                                    void* hip_stream) {
  if (!fam || !gal) return fail(GFC_EINVAL, "null Sersic family or galaxy block");
  if (fam->ctx != ctx) return fail(GFC_EINVAL, "Sersic family belongs to another context");
  if (n > 0 && !sersic_n) return fail(GFC_EINVAL, "null Sersic index array");
  if (gal->mix_id) return fail(GFC_EINVAL, "mix_id is not used with a Sersic family (pass NULL)");
  // a stand-in for the mixture argument: only its context is read before the tables are replaced
  gfc_mix shell;
  shell.ctx = ctx;
  shell.n_tables = 1;
  shell.kmax = fam->K;
  hipStream_t s = (hipStream_t)hip_stream;
  const int S = fam->S, K = fam->K;
  const float* grid = fam->d_grid;
  return render_per_galaxy(ctx, psf, &shell, K, gal, n, W, flags, out, s, [&](PerGalaxyTables t) {
    hipLaunchKernelGGL(sersic_tables_kernel, dim3(table_blocks(n)), dim3(kPre), 0, s,
                       sersic_n, S, grid, K, n, t);
    return hipGetLastError();
  });
}

gfc_status gfc_render_stamps_composite(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, int disk_table,
                                       int bulge_table, const gfc_galaxies* gal, const float* bulge_frac,
                                       const float* bulge_rho, int64_t n, int W, unsigned flags, float* out,
                                       void* hip_stream) {
  if (!mix || !gal) return fail(GFC_EINVAL, "null mixture or galaxy block");
  if (disk_table < 0 || disk_table >= mix->n_tables || bulge_table < 0 || bulge_table >= mix->n_tables)
    return fail(GFC_EINVAL, "disk or bulge table out of range");
  if (n > 0 && (!bulge_frac || !bulge_rho)) return fail(GFC_EINVAL, "null bulge fraction or radius ratio");
  if (gal->mix_id) return fail(GFC_EINVAL, "mix_id is not used with a composite (pass NULL)");
  const int Kd = mix->K[disk_table], Kb = mix->K[bulge_table];
  if (Kd + Kb > kKmax) return fail(GFC_EINVAL, "disk and bulge together exceed 16 components");
  hipStream_t s = (hipStream_t)hip_stream;
  const float* mamp = mix->d_amp;
  const float* mvar = mix->d_var;
  return render_per_galaxy(ctx, psf, mix, Kd + Kb, gal, n, W, flags, out, s, [&](PerGalaxyTables t) {
    hipLaunchKernelGGL(composite_tables_kernel, dim3(table_blocks(n)), dim3(kPre), 0, s,
                       mamp, mvar, disk_table, Kd, bulge_table, Kb, bulge_frac, bulge_rho, n, t);
    return hipGetLastError();
  });
}

}  // extern "C"
