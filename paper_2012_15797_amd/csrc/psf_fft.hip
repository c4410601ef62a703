// PSF spectrum for the PSF-FT cache (Lang 2020, Section 2, steps 1-2).
//
// Cold path: computed once per (PSF, stamp size).  A separable DFT in float64
// with exactly reduced phase indices, rounded once to float32:
//   P_hat[k_y][k_x] = sum_{r,c} P[r][c] exp(-2 pi i (k_x (c - S_x/2) + k_y (r - S_y/2)) / W).
// Writing the phase with (c - S_x/2) mod W folds the S_y x S_x grid onto the
// W x W grid periodically with the centre pixel at index 0 (zero padding when
// W >= S).
#include "gfc_launch.hpp"

namespace gfc {

__device__ __forceinline__ int pmod(int a, int m) {
  const int r = a % m;
  return r < 0 ? r + m : r;
}

// tmp[r][kx] = sum_c P[r][c] exp(-2 pi i kx (c - Sx/2) / W),  kx = 0..W/2
__global__ void psf_row_dft(const double* __restrict__ pix, int Sy, int Sx, int W,
                            double2* __restrict__ tmp) {
  const int H = W / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Sy * H) return;
  const int r = idx / H, kx = idx % H;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < Sx; ++c) {
    const int ph = (int)(((int64_t)kx * pmod(c - Sx / 2, W)) % W);
    double s, co;
    sincospi(-2.0 * (double)ph / (double)W, &s, &co);
    const double v = pix[(int64_t)r * Sx + c];
    re = fma(v, co, re);
    im = fma(v, s, im);
  }
  tmp[idx] = make_double2(re, im);
}

// P_hat[ky][kx] = sum_r tmp[r][kx] exp(-2 pi i ky (r - Sy/2) / W)
__global__ void psf_col_dft(const double2* __restrict__ tmp, int Sy, int W,
                            float2* __restrict__ main_cols, float2* __restrict__ nyq_col,
                            float2* __restrict__ natural) {
  const int H = W / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= W * H) return;
  const int ky = idx / H, kx = idx % H;
  double re = 0.0, im = 0.0;
  for (int r = 0; r < Sy; ++r) {
    const int ph = (int)(((int64_t)ky * pmod(r - Sy / 2, W)) % W);
    double s, co;
    sincospi(-2.0 * (double)ph / (double)W, &s, &co);
    const double2 t = tmp[(int64_t)r * H + kx];
    re += t.x * co - t.y * s;
    im += t.x * s + t.y * co;
  }
  const float2 v = make_float2((float)re, (float)im);
  if (kx < W / 2) {
    // Lane-permuted for the render kernels: lane (c = kx, h = ky mod D) of a
    // stamp reads element (ky / D) * (D W / 2) + D kx + h, where D is the
    // decimation of the column transform (4 for W = 256, 2 otherwise).
    const int D = (W == 256) ? 4 : 2;
    main_cols[(ky / D) * (D * (W / 2)) + D * kx + (ky % D)] = v;
  } else {
    nyq_col[ky] = v;
  }
  if (natural) natural[idx] = v;
}

hipError_t launch_psf_spectrum(const double* pix, int Sy, int Sx, int W, double2* tmp,
                               float2* main_cols, float2* nyq_col, float2* natural,
                               hipStream_t stream) {
  const int H = W / 2 + 1;
  const int n1 = Sy * H, n2 = W * H;
  hipLaunchKernelGGL(psf_row_dft, dim3((n1 + 255) / 256), dim3(256), 0, stream, pix, Sy, Sx, W, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psf_col_dft, dim3((n2 + 255) / 256), dim3(256), 0, stream, tmp, Sy, W,
                     main_cols, nyq_col, natural);
  return hipGetLastError();
}

}  // namespace gfc
