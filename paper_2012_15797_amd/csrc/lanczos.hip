// Lanczos sub-pixel shift of finished stamps (Lang 2020, Section 2, step 8:
// the optional pixel-space alternative to the Fourier phase).  With
// GFC_SHIFT_LANCZOS3 the render places each galaxy at the integer part of its
// position; this pass then shifts the whole stamp, real-space terms included,
// by the fractional part:
//   out[r][c] = sum_{dy,dx = -3..2} wy[dy] wx[dx] in[r + dy][c + dx],
//   w[d] = L(d + f) / sum_d' L(d' + f),  L(t) = sinc(t) sinc(t / 3) on |t| < 3,
// with pixels outside the stamp taken as zero.  Separable: rows, then columns.
//
// This pass serves W = 128 and 256 (up to 64 x 64 the render kernel applies
// the same filter while it stores): one read and one write of the stamp,
// in place.
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

namespace gfc {

namespace {

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

// One workgroup of W threads per stamp, thread c owning column c.  It walks
// down the stamp's rows once: row r is loaded (coalesced) and filtered along
// x through a double-buffered LDS row with three zero pixels on each side;
// the six most recent x-filtered rows stay in registers, and output row
// r - 2 (taps r - 5 .. r) is stored as soon as row r is in.  The pass is in
// place: a row is overwritten only after every thread has read it.  LDS is
// two rows, so many workgroups share a CU and hide the memory latency.
template <int W>
__global__ void __launch_bounds__(W) lanczos_stream_kernel(const float* __restrict__ x,
                                                           const float* __restrict__ y, float* out) {
  constexpr int PAD = 3;                 // zero pixels on each side of a row
  __shared__ float row[2][W + 2 * PAD];
  __shared__ float s_w[12];
  const int64_t s = blockIdx.x;
  float* img = out + s * (int64_t)(W * W);
  float wx[6], wy[6];
  block_weights(x[s], y[s], s_w, wx, wy);
  const int c = threadIdx.x;
  if (c < 2 * PAD) {  // the margins of both buffers
    const int col = c < PAD ? c : W + c;
    row[0][col] = 0.f;
    row[1][col] = 0.f;
  }
  float hw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // x-filtered rows r - 5 .. r
  float next = img[c];
  for (int r = 0; r < W + 2; ++r) {
    float h = 0.f;
    if (r < W) {  // uniform
      const float v = next;
      if (r + 1 < W) next = img[(r + 1) * W + c];  // in flight during this row
      float* b = row[r & 1];
      b[PAD + c] = v;
      __syncthreads();
#pragma unroll
      for (int d = 0; d < 6; ++d) h = fmaf(wx[d], b[c + d], h);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) hw[i] = hw[i + 1];
    hw[5] = h;
    if (r >= 2) {
      float o = 0.f;
#pragma unroll
      for (int j = 0; j < 6; ++j) o = fmaf(wy[j], hw[j], o);
      __builtin_nontemporal_store(o, &img[(r - 2) * W + c]);
    }
  }
}

}  // namespace

hipError_t launch_lanczos_shift(const RenderArgs& a, int W, hipStream_t stream) {
  constexpr int64_t kMaxBlocks = (int64_t)1 << 30;
  for (int64_t done = 0; done < a.n;) {
    const int64_t chunk = std::min<int64_t>(a.n - done, kMaxBlocks);
    const float* x = a.x + done;
    const float* y = a.y + done;
    float* o = a.out + done * (int64_t)W * W;
    switch (W) {
      case 128: hipLaunchKernelGGL(lanczos_stream_kernel<128>, dim3((unsigned)chunk), dim3(128), 0, stream, x, y, o); break;
      case 256: hipLaunchKernelGGL(lanczos_stream_kernel<256>, dim3((unsigned)chunk), dim3(256), 0, stream, x, y, o); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace gfc
