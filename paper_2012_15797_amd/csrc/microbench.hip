// Rate probes for the roofline denominators (include/gfc_microbench.h).
//
// Each ALU probe launches 2,048 workgroups of 256 threads (8 wavefronts per
// SIMD on 256 CUs) whose lanes run independent dependency chains, enough to
// hide every latency, so the time measures issue rate alone.  The results
// feed a sink only when they take an impossible value, which keeps the
// arithmetic live without a store per lane.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "gfc_microbench.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));  // native vector (the nontemporal builtins take it)

constexpr int kBlock = 256;
constexpr int kGrid = 2048;
constexpr int kFmaIters = 4096;   // x 16 chains: 65,536 FMAs per lane
constexpr int kExpIters = 1024;   // x 16 chains: 16,384 exponentials per lane
constexpr int kMixIters = 1024;   // x 8 groups

__global__ void __launch_bounds__(kBlock) fma_probe(float b, float c, float* sink) {
  float a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = (float)(threadIdx.x + i) * 1e-3f;
  for (int it = 0; it < kFmaIters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = fmaf(a[i], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += a[i];
  if (s == -FLT_MAX) sink[0] = s;
}

__global__ void __launch_bounds__(kBlock) exp_probe(float* sink) {
  float x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = (float)(threadIdx.x + i) * 1e-3f;
  for (int it = 0; it < kExpIters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = __builtin_amdgcn_exp2f(-x[i]);  // converges to ~0.64
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += x[i];
  if (s == -FLT_MAX) sink[0] = s;
}

// Per step and group g: x_g <- exp2(-x_g), and F FMAs y_gj <- y_gj b + c on
// accumulators of their own (independent of the exponentials).
template <int F>
__global__ void __launch_bounds__(kBlock) exp_fma_probe(float b, float c, float* sink) {
  constexpr int G = 8;
  float x[G];
  float y[G][F > 0 ? F : 1];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    x[g] = (float)(threadIdx.x + g) * 1e-3f;
#pragma unroll
    for (int j = 0; j < (F > 0 ? F : 1); ++j) y[g][j] = (float)(g + j) * 1e-3f;
  }
  for (int it = 0; it < kMixIters; ++it) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      x[g] = __builtin_amdgcn_exp2f(-x[g]);
#pragma unroll
      for (int j = 0; j < F; ++j) y[g][j] = fmaf(y[g][j], b, c);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    s += x[g];
#pragma unroll
    for (int j = 0; j < F; ++j) s += y[g][j];
  }
  if (s == -FLT_MAX) sink[0] = s;
}

__global__ void __launch_bounds__(kBlock) write_probe(v4f* __restrict__ dst, int64_t n4) {
  const v4f v = {1.f, 2.f, 3.f, 4.f};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock)
    __builtin_nontemporal_store(v, &dst[i]);
}

__global__ void __launch_bounds__(kBlock) copy_probe(v4f* __restrict__ dst, const v4f* __restrict__ src,
                                                     int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock)
    __builtin_nontemporal_store(src[i], &dst[i]);
}

// One untimed launch, then reps timed ones; the shortest time in seconds.
template <typename Launch>
int timed(int reps, hipStream_t s, Launch launch, double* best_s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  double best = 1e30;
  for (int r = 0; r < (reps > 0 ? reps : 1) && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
    launch();
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms > 0.f && ms * 1e-3 < best) best = ms * 1e-3;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return -(int)e;
  *best_s = best;
  return 0;
}

constexpr double kLanes = (double)kGrid * kBlock;

int streaming_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return cus * 8;
}

}  // namespace

extern "C" {

int gfc_mb_fma(int reps, float* sink, void* hip_stream, double* lane_fma_per_s) {
  hipStream_t s = (hipStream_t)hip_stream;
  double t = 0;
  const int rc = timed(reps, s, [&] {
    hipLaunchKernelGGL(fma_probe, dim3(kGrid), dim3(kBlock), 0, s, 0.9999f, 1e-4f, sink);
  }, &t);
  if (rc == 0) *lane_fma_per_s = kLanes * kFmaIters * 16.0 / t;
  return rc;
}

int gfc_mb_exp(int reps, float* sink, void* hip_stream, double* lane_exp_per_s) {
  hipStream_t s = (hipStream_t)hip_stream;
  double t = 0;
  const int rc = timed(reps, s, [&] {
    hipLaunchKernelGGL(exp_probe, dim3(kGrid), dim3(kBlock), 0, s, sink);
  }, &t);
  if (rc == 0) *lane_exp_per_s = kLanes * kExpIters * 16.0 / t;
  return rc;
}

int gfc_mb_exp_fma(int fma_per_exp, int reps, float* sink, void* hip_stream, double* lane_exp_per_s,
                   double* lane_fma_per_s) {
  hipStream_t s = (hipStream_t)hip_stream;
  double t = 0;
  int rc = -(int)hipErrorInvalidValue;
  auto run = [&](auto kernel) {
    rc = timed(reps, s, [&] {
      hipLaunchKernelGGL(kernel, dim3(kGrid), dim3(kBlock), 0, s, 0.9999f, 1e-4f, sink);
    }, &t);
  };
  switch (fma_per_exp) {
    case 0: run(exp_fma_probe<0>); break;
    case 1: run(exp_fma_probe<1>); break;
    case 2: run(exp_fma_probe<2>); break;
    case 3: run(exp_fma_probe<3>); break;
    case 4: run(exp_fma_probe<4>); break;
    case 6: run(exp_fma_probe<6>); break;
    case 8: run(exp_fma_probe<8>); break;
    default: return rc;
  }
  if (rc == 0) {
    const double steps = kLanes * kMixIters * 8.0;
    *lane_exp_per_s = steps / t;
    *lane_fma_per_s = steps * fma_per_exp / t;
  }
  return rc;
}

int gfc_mb_hbm_write(float* dst, size_t bytes, int reps, void* hip_stream, double* bytes_per_s) {
  if (!dst || bytes == 0 || (bytes & 15)) return -(int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n4 = (int64_t)(bytes / 16);
  const int grid = streaming_grid();
  double t = 0;
  const int rc = timed(reps, s, [&] {
    hipLaunchKernelGGL(write_probe, dim3(grid), dim3(kBlock), 0, s, reinterpret_cast<v4f*>(dst), n4);
  }, &t);
  if (rc == 0) *bytes_per_s = (double)bytes / t;
  return rc;
}

int gfc_mb_hbm_copy(float* dst, const float* src, size_t bytes, int reps, void* hip_stream, double* bytes_per_s) {
  if (!dst || !src || bytes == 0 || (bytes & 15)) return -(int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n4 = (int64_t)(bytes / 16);
  const int grid = streaming_grid();
  double t = 0;
  const int rc = timed(reps, s, [&] {
    hipLaunchKernelGGL(copy_probe, dim3(grid), dim3(kBlock), 0, s, reinterpret_cast<v4f*>(dst),
                       reinterpret_cast<const v4f*>(src), n4);
  }, &t);
  if (rc == 0) *bytes_per_s = 2.0 * (double)bytes / t;
  return rc;
}

}  // extern "C"
