// Lanczos sub-pixel shift of finished stamps (Lang 2020, Section 2, step 8:
// the optional pixel-space alternative to the Fourier phase).  With
// GFC_SHIFT_LANCZOS3 the render places each galaxy at the integer part of its
// position; this pass then shifts the whole stamp, real-space terms included,
// by the fractional part:
//   out[r][c] = sum_{dy,dx = -3..2} wy[dy] wx[dx] in[r + dy][c + dx],
//   w[d] = L(d + f) / sum_d' L(d' + f),  L(t) = sinc(t) sinc(t / 3) on |t| < 3,
// with pixels outside the stamp taken as zero.  Separable: rows, then columns.
//
// These passes serve W = 128 and 256 (up to 64 x 64 the render kernel
// applies the same filter while it stores).  W = 128: one workgroup per
// stamp, the stamp held in LDS, both passes in place, one read and one write
// of the stamp.  W = 256 (256 KB per stamp): a row-band pass and a
// column-band pass, each in place through LDS.
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

namespace gfc {

namespace {

constexpr int kThreads = 256;

// Fills w[0..5] (taps d = -3..2) for the fractional part of v; lanes 0..11 of
// the block compute the raw values, every lane normalises.
__device__ __forceinline__ void block_weights(float vx, float vy, float* s_w, float (&wx)[6], float (&wy)[6]) {
  const int t = threadIdx.x;
  if (t < 12) {
    const float v = t < 6 ? vx : vy;
    const float f = v - floorf(v);
    s_w[t] = lanczos3((float)((t % 6) - 3) + f);
  }
  __syncthreads();
  float sx = 0.f, sy = 0.f;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    wx[d] = s_w[d];
    wy[d] = s_w[6 + d];
    sx += wx[d];
    sy += wy[d];
  }
  const float rx = 1.f / sx, ry = 1.f / sy;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    wx[d] *= rx;
    wy[d] *= ry;
  }
}

template <int W>
__global__ void __launch_bounds__(kThreads) lanczos_tile_kernel(const float* __restrict__ x,
                                                                const float* __restrict__ y, float* out) {
  constexpr int TS = W + 1;
  constexpr int PER = W * W / kThreads;  // pixels per thread
  static_assert(W * W % kThreads == 0, "stamp size");
  __shared__ float tile[W * TS];
  __shared__ float s_w[12];
  const int64_t s = blockIdx.x;
  float* img = out + s * (int64_t)(W * W);
  float wx[6], wy[6];
  block_weights(x[s], y[s], s_w, wx, wy);
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = t + k * kThreads;
    tile[(i / W) * TS + (i % W)] = img[i];
  }
  __syncthreads();
  float hv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = t + k * kThreads, r = i / W, c = i % W;
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int cc = c + d - 3;
      if (cc >= 0 && cc < W) acc = fmaf(wx[d], tile[r * TS + cc], acc);
    }
    hv[k] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = t + k * kThreads;
    tile[(i / W) * TS + (i % W)] = hv[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = t + k * kThreads, r = i / W, c = i % W;
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int rr = r + d - 3;
      if (rr >= 0 && rr < W) acc = fmaf(wy[d], tile[rr * TS + c], acc);
    }
    __builtin_nontemporal_store(acc, &img[i]);
  }
}

// W = 256: BAND rows (or columns) of one stamp per workgroup.
constexpr int kW = 256;
constexpr int BAND = 16;

__global__ void __launch_bounds__(kThreads) lanczos_rows_kernel(const float* __restrict__ x,
                                                                const float* __restrict__ y, float* out) {
  __shared__ float tile[BAND * kW];
  __shared__ float s_w[12];
  const int64_t s = blockIdx.x / (kW / BAND);
  const int r0 = (blockIdx.x % (kW / BAND)) * BAND;
  float* img = out + s * (int64_t)(kW * kW) + r0 * kW;
  float wx[6], wy[6];
  block_weights(x[s], y[s], s_w, wx, wy);
  const int t = threadIdx.x;  // = column
#pragma unroll
  for (int r = 0; r < BAND; ++r) tile[r * kW + t] = img[r * kW + t];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < BAND; ++r) {
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int cc = t + d - 3;
      if (cc >= 0 && cc < kW) acc = fmaf(wx[d], tile[r * kW + cc], acc);
    }
    img[r * kW + t] = acc;
  }
}

__global__ void __launch_bounds__(kThreads) lanczos_cols_kernel(const float* __restrict__ x,
                                                                const float* __restrict__ y, float* out) {
  constexpr int TS = BAND + 1;
  __shared__ float tile[kW * TS];
  __shared__ float s_w[12];
  const int64_t s = blockIdx.x / (kW / BAND);
  const int c0 = (blockIdx.x % (kW / BAND)) * BAND;
  float* img = out + s * (int64_t)(kW * kW) + c0;
  float wx[6], wy[6];
  block_weights(x[s], y[s], s_w, wx, wy);
  const int t = threadIdx.x;
  const int cl = t % BAND, rq = t / BAND;  // 16 columns x 16 row phases
#pragma unroll
  for (int k = 0; k < kW / (kThreads / BAND); ++k) {
    const int r = rq + k * (kThreads / BAND);
    tile[r * TS + cl] = img[r * kW + cl];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kW / (kThreads / BAND); ++k) {
    const int r = rq + k * (kThreads / BAND);
    float acc = 0.f;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int rr = r + d - 3;
      if (rr >= 0 && rr < kW) acc = fmaf(wy[d], tile[rr * TS + cl], acc);
    }
    __builtin_nontemporal_store(acc, &img[r * kW + cl]);
  }
}

}  // namespace

hipError_t launch_lanczos_shift(const RenderArgs& a, int W, hipStream_t stream) {
  constexpr int64_t kMaxBlocks = (int64_t)1 << 30;
  for (int64_t done = 0; done < a.n;) {
    const int64_t per = (W == kW) ? (kW / BAND) : 1;  // workgroups per stamp
    const int64_t chunk = std::min<int64_t>(a.n - done, kMaxBlocks / per);
    const float* x = a.x + done;
    const float* y = a.y + done;
    float* o = a.out + done * (int64_t)W * W;
    const dim3 grid((unsigned)(chunk * per)), block(kThreads);
    switch (W) {
      case 128: hipLaunchKernelGGL(lanczos_tile_kernel<128>, grid, block, 0, stream, x, y, o); break;
      case 256:
        hipLaunchKernelGGL(lanczos_rows_kernel, grid, block, 0, stream, x, y, o);
        hipLaunchKernelGGL(lanczos_cols_kernel, grid, block, 0, stream, x, y, o);
        break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace gfc
