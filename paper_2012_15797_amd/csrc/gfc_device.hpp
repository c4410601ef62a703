// Device-side shared definitions of the renderer: kernel argument blocks and
// the per-galaxy shape algebra (Section 2, steps 3 and 4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_reg.hpp"

namespace gfc {

constexpr int kKmax = 16;
// -2 pi^2 log2(e): the Gaussian transform exp(-2 pi^2 q) written as exp2(kQ q).
constexpr float kQ = -0x1.c7a47ep+4f;
// -log2(e) / 2: a real-space Gaussian exp(-u^T S^-1 u / 2) as exp2(kHalfLog2e q).
constexpr float kHalfLog2e = -0x1.715476p-1f;
constexpr float kInv2Pi = 0x1.45f306p-3f;

// Galaxy parameters and everything a render launch needs.
struct RenderArgs {
  const float* x;
  const float* y;
  const float* flux;
  const float* r_e;
  const float* e1;
  const float* e2;
  const int32_t* mix_id;   // may be null (table 0)
  const float* amp;        // [n_tables][kKmax]
  const float* var;        // [n_tables][kKmax]
  const int32_t* K;        // [n_tables]
  int n_tables;
  int kmax;                // max K over the tables
  float cdinv[4];          // CD^{-1}, row-major (identity by default)
  float pg[6];             // PSF Gaussian: mu_x, mu_y, c_xx, c_xy, c_yy, amp
  const float2* psf_main;  // PSF spectrum, lane-permuted columns 0..W/2-1
  const float2* psf_nyq;   // PSF spectrum, Nyquist column k_x = W/2, [W]
  float* out;              // [n][W][W]
  int64_t n;
  unsigned flags;
  unsigned long long* invalid;  // device counter of invalid galaxies
  // Spatially varying (eigen-)PSF; eig_J == 0 for a constant PSF.
  int eig_J;                // components; their spectra follow each other eig_stride float2 apart
  int eig_degree;           // polynomial degree (0..3)
  int64_t eig_stride;
  const float* eig_coef;    // [J][T], T = (degree + 1)(degree + 2) / 2
  const float* eig_mom;     // [J][6]: sum, sum x, sum y, sum x^2, sum x y, sum y^2 about the centre pixel
  float eig_norm[4];        // x_off, 1 / x_scale, y_off, 1 / y_scale
  const float* psf_px;      // [n] image position of each galaxy (eigen PSF only)
  const float* psf_py;
  // Stamps of several constant PSFs in one launch (serving): galaxy i uses
  // PSF psf_id[i] of these tables instead of psf_main / psf_nyq / pg.  An
  // index outside [0, n_psf) makes the galaxy invalid.  Null psf_id: one PSF.
  const int32_t* psf_id;              // [n]
  const float2* const* psf_main_tab;  // [n_psf] spectra for this W, laid out as psf_main
  const float2* const* psf_nyq_tab;   // [n_psf] Nyquist columns
  const float* pg_tab;                // [n_psf][6] PSF Gaussians
  int n_psf;
};

constexpr int kEigMax = 16;     // eigen-PSF components
constexpr int kEigDegMax = 3;   // polynomial degree

enum : unsigned { kForceFourier = 1u, kForceReal = 2u, kRampLinear = 4u, kLanczos3 = 8u, kAccumulate = 16u };

// Per-galaxy state shared by every step.
struct Galaxy {
  float x0, y0, flux;
  float fx, fy;      // fractional centre (in [0, 1))
  int nx, ny;        // integer centre modulo W
  float b11, b12, b22;  // pixel-space covariance per unit mixture variance
  int table, K;
  bool ok;
};

__device__ __forceinline__ bool finitef(float v) { return __builtin_isfinite(v); }

// Step 3: C_i = v_i B with B = A A^T, A = CD^{-1} E.  With c^2, s^2 and cs of
// the position angle written through e1, e2 (Appendix A), E E^T is
// r_e^2/(1+e)^2 [[1+e^2-2e1, 2e2], [2e2, 1+e^2+2e1]] -- no trigonometry.
// A galaxy's inputs as they are stored.
struct GalaxyIn {
  float x, y, flux, re, e1, e2;
  int table;
};

__device__ __forceinline__ GalaxyIn load_galaxy_in(const RenderArgs& p, int64_t g) {
  return GalaxyIn{p.x[g], p.y[g], p.flux[g], p.r_e[g], p.e1[g], p.e2[g], p.mix_id ? p.mix_id[g] : 0};
}

template <int W>
__device__ __forceinline__ Galaxy make_galaxy(const RenderArgs& p, const GalaxyIn& in) {
  Galaxy G;
  G.x0 = in.x;
  G.y0 = in.y;
  G.flux = in.flux;
  const float re = in.re, e1 = in.e1, e2 = in.e2;
  // The table follows from mix_id alone (an index out of range takes table
  // 0 and makes the galaxy invalid), so its reads need not wait for the
  // other parameters.
  const bool table_ok = in.table >= 0 && in.table < p.n_tables;
  G.table = table_ok ? in.table : 0;
  G.K = p.K[G.table];
  const float esq = e1 * e1 + e2 * e2;
  G.ok = finitef(G.x0) && finitef(G.y0) && finitef(G.flux) && finitef(re) && finitef(e1) &&
         finitef(e2) && re > 0.f && esq < 1.f && fabsf(G.x0) <= 8388608.f &&
         fabsf(G.y0) <= 8388608.f && table_ok;
  // An invalid galaxy renders as NaN everywhere: a NaN flux propagates
  // through every product of the Fourier and real-space paths.
  if (!G.ok) G.flux = __builtin_nanf("");
  const float fxf = floorf(G.x0), fyf = floorf(G.y0);
  if (p.flags & kLanczos3) {  // rendered at the integer position; the stamp is shifted afterwards
    G.x0 = fxf;
    G.y0 = fyf;
  }
  G.fx = G.ok ? G.x0 - fxf : 0.f;
  G.fy = G.ok ? G.y0 - fyf : 0.f;
  G.nx = G.ok ? ((int)(fxf - (float)W * floorf(fxf * (1.f / W)))) & (W - 1) : 0;
  G.ny = G.ok ? ((int)(fyf - (float)W * floorf(fyf * (1.f / W)))) & (W - 1) : 0;
  // Hardware square root and reciprocal (about 1 ulp each): the covariance
  // needs no correctly rounded operations, and these are a few instructions
  // instead of some thirty.
  const float e = __builtin_amdgcn_sqrtf(esq);
  const float s = (re * re) * __builtin_amdgcn_rcpf((1.f + e) * (1.f + e));
  const float c11 = s * (1.f + esq - 2.f * e1);
  const float c12 = s * (2.f * e2);
  const float c22 = s * (1.f + esq + 2.f * e1);
  // B = M C M^T with M = CD^{-1}
  const float m00 = p.cdinv[0], m01 = p.cdinv[1], m10 = p.cdinv[2], m11 = p.cdinv[3];
  const float p00 = fmaf(m00, c11, m01 * c12), p01 = fmaf(m00, c12, m01 * c22);
  const float p10 = fmaf(m10, c11, m11 * c12), p11 = fmaf(m10, c12, m11 * c22);
  G.b11 = fmaf(p00, m00, p01 * m01);
  G.b12 = fmaf(p00, m10, p01 * m11);
  G.b22 = fmaf(p10, m10, p11 * m11);
  return G;
}

template <int W>
__device__ __forceinline__ Galaxy load_galaxy(const RenderArgs& p, int64_t g) {
  return make_galaxy<W>(p, load_galaxy_in(p, g));
}

// Fourier bins where a component's exponent (log2 of its share of the
// component's amplitude) is below -kSkipLog2 may be skipped: every skipped
// value is below 2^-40 of the amplitude, far under FP32 rounding of the stamp.
constexpr float kSkipLog2 = 40.f;

// A lower bound on the smallest eigenvalue of the galaxy's shape matrix B,
// so that q(nu, omega) >= lambda (nu^2 + omega^2): the eigenvalue of the
// FP32 matrix in double precision (no cancellation at any ellipticity),
// less 0.1 per cent.
__device__ __forceinline__ float shape_min_eig(const Galaxy& G) {
  const double a = G.b11, b = G.b12, d = G.b22;
  const double h = 0.5 * (a - d);
  const double lam = 0.5 * (a + d) - sqrt(h * h + b * b);
  return lam > 0.0 ? (float)(0.999 * lam) : 0.f;
}

// A kernel's first argument A, read through a pointer that is renewed
// opaquely at each call: its fields are reloaded through the scalar cache
// there instead of being held in registers from the kernel's start (inside
// a persistent loop, or late in a long kernel).
template <typename A>
__device__ __forceinline__ const A& kernel_args_renewed() {
  typedef const __attribute__((address_space(4))) A* KArgs;
  KArgs pk = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(pk));
  return *(const A*)pk;
}

__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// For a wavefront (or workgroup) that renders one stamp: the galaxy's values
// are the same in every lane, so they move to scalar registers.  This frees
// vector registers and turns the mixture-table reads into scalar loads.
__device__ __forceinline__ void make_uniform(Galaxy& G) {
  G.x0 = uniform_f(G.x0);
  G.y0 = uniform_f(G.y0);
  G.flux = uniform_f(G.flux);
  G.fx = uniform_f(G.fx);
  G.fy = uniform_f(G.fy);
  G.nx = __builtin_amdgcn_readfirstlane(G.nx);
  G.ny = __builtin_amdgcn_readfirstlane(G.ny);
  G.b11 = uniform_f(G.b11);
  G.b12 = uniform_f(G.b12);
  G.b22 = uniform_f(G.b22);
  G.table = __builtin_amdgcn_readfirstlane(G.table);
  G.K = __builtin_amdgcn_readfirstlane(G.K);
  G.ok = __builtin_amdgcn_readfirstlane((int)G.ok) != 0;
}

// Weight of eigen-PSF component j at normalised position (u, v): the sum
// over polynomial terms u^a v^b (a + b <= degree, ordered by the power of v,
// then of u) of the component's coefficients.  up/vp hold powers 0..3.
__device__ __forceinline__ float eigen_weight(const RenderArgs& p, int j, const float (&up)[kEigDegMax + 1],
                                              const float (&vp)[kEigDegMax + 1]) {
  const int D = p.eig_degree;
  const float* cf = p.eig_coef + j * ((D + 1) * (D + 2) / 2);
  float c = 0.f;
  static_for<0, kEigDegMax + 1>([&](auto bb) {
    constexpr int b = decltype(bb)::value;
    static_for<0, kEigDegMax + 1 - b>([&](auto aa) {
      constexpr int a = decltype(aa)::value;
      if (a + b <= D) c = fmaf(cf[b * (D + 1) - b * (b - 1) / 2 + a], up[a] * vp[b], c);
    });
  });
  return c;
}

// The PSF Gaussian {mu_x, mu_y, c_xx, c_xy, c_yy, amp} of the weighted sum
// of components: moments are linear in the weights.
__device__ __forceinline__ void eigen_gauss(const float (&mom)[6], float (&pg)[6]) {
  const float F = mom[0], rF = 1.f / F;
  const float mx = mom[1] * rF, my = mom[2] * rF;
  pg[0] = mx;
  pg[1] = my;
  pg[2] = fmaf(mom[3], rF, -mx * mx);
  pg[3] = fmaf(mom[4], rF, -mx * my);
  pg[4] = fmaf(mom[5], rF, -my * my);
  pg[5] = F;
}

// (sin(pi r), cos(pi r)) for |r| < 2^22, without the special-value handling
// of the library routine.  r = j/2 + f with j = rint(2 r) and |f| <= 1/4 (f is
// exact); sin(pi f) and cos(pi f) are their Taylor series through f^9 and
// f^10 (truncation below 2e-9 on |f| <= 1/4), and j mod 4 picks the quadrant.
GFC_HD void sincospi_poly(float r, float* s_out, float* c_out) {
  const float j = rintf(2.f * r);
  const float f = fmaf(-0.5f, j, r);
  const float f2 = f * f;
  float sp = fmaf(f2, 0x1.5078340p-4f, -0x1.32d2ccp-1f);  // pi^9/9!, -pi^7/7!
  sp = fmaf(f2, sp, 0x1.466bc6p+1f);                      // pi^5/5!
  sp = fmaf(f2, sp, -0x1.4abbcep+2f);                     // -pi^3/3!
  sp = fmaf(f2, sp, 0x1.921fb6p+1f) * f;                  // pi
  float cp = fmaf(f2, -0x1.a6d1f2p-6f, 0x1.e1f506p-3f);   // -pi^10/10!, pi^8/8!
  cp = fmaf(f2, cp, -0x1.55d3c8p+0f);                     // -pi^6/6!
  cp = fmaf(f2, cp, 0x1.03c1f0p+2f);                      // pi^4/4!
  cp = fmaf(f2, cp, -0x1.3bd3ccp+2f);                     // -pi^2/2!
  cp = fmaf(f2, cp, 1.f);
  const int q = (int)j;
  const float s = (q & 1) ? cp : sp;
  const float c = (q & 1) ? sp : cp;
  *s_out = __builtin_bit_cast(float, __builtin_bit_cast(int, s) ^ ((q & 2) << 30));
  *c_out = __builtin_bit_cast(float, __builtin_bit_cast(int, c) ^ (((q + 1) & 2) << 30));
}

// The value held by the even lane of this lane's pair (DPP quad permute
// 0, 0, 2, 2).
__device__ __forceinline__ float pair_even(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xA0, 0xF, 0xF, false));
}

// The value held by the second lane of this lane's stamp, for stamps of W
// consecutive lanes (W >= 64: lane 1 of the wavefront).
template <int W>
__device__ __forceinline__ float stamp_lane1(float v) {
  if constexpr (W >= 64) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 1));
  } else {
    return __shfl(v, ((int)__lane_id() & ~(W - 1)) + 1, 64);
  }
}

// Value of v in lane k of the wavefront (k uniform).
__device__ __forceinline__ float lane_f(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// Raw Lanczos-3 value at t (exact zeros at the integers other than 0), for
// the optional pixel-space sub-pixel shift (Section 2, step 8).
__device__ __forceinline__ float lanczos3(float t) {
  if (t == 0.f) return 1.f;
  if (fabsf(t) >= 3.f || t == rintf(t)) return 0.f;
  const float s = sinpif(t) * sinpif(t * (1.f / 3.f));
  return s * (3.f * 0.10132118364233778f) / (t * t);  // sinc(t) sinc(t/3) = 3 sin(pi t) sin(pi t/3) / (pi t)^2
}

// Step 4: Fourier weight of a component whose covariance trace is `tr`.
template <int W>
__device__ __forceinline__ float route_weight(float tr, unsigned flags) {
  if (flags & kForceFourier) return 1.f;
  if (flags & kForceReal) return 0.f;
  const float n = (0.5f * (float)W) * __builtin_amdgcn_rsqf(tr);
  const float t = fminf(fmaxf(n - 3.f, 0.f), 1.f);
  if (flags & kRampLinear) return t;
  return t * t * (3.f - 2.f * t);
}

// d w / d n of route_weight (zero outside the ramp).
template <int W>
__device__ __forceinline__ float route_slope(float n, unsigned flags) {
  if (flags & (kForceFourier | kForceReal)) return 0.f;
  if (!(n > 3.f && n < 4.f)) return 0.f;
  const float t = n - 3.f;
  if (flags & kRampLinear) return 1.f;
  return 6.f * t * (1.f - t);
}

}  // namespace gfc
