// Forward render kernel for 256 x 256 stamps (Lang 2020, Section 2, steps
// 3-8): one 1,024-thread workgroup per stamp, the whole half spectrum kept
// on the chip, in registers and LDS.  Nothing but the stamp goes to memory.
//
//  column phase    lane (c, h), c = 0..127, h = 0..7, evaluates the mixture
//                  transform on column k_x = c, rows k_y = 8m + h (steps
//                  5-6), applies the shift phase, the flux and the cached PSF
//                  spectrum (step 7a), and runs a 32-point inverse FFT in
//                  registers.  Both integer parts of the centre enter the
//                  phase as exact table entries, so the stamp leaves the
//                  transforms in output order (no roll).  Column k_x = 128 is
//                  packed into column 0 as its imaginary part: both columns
//                  transform to real vectors.
//  column combine  the radix-8 stage of the 256-point column transform across
//                  the eight lanes of a column, through a slice of LDS that
//                  only its wavefront uses (no workgroup barrier).  Lane
//                  (c, h) ends with the rows y = h (mod 8) of column c: 16 in
//                  each half of the stamp.
//  row phase       per half (128 rows): the column values go to LDS row-major
//                  (135 KB); eight lanes per row run the complex-to-real row
//                  transform (the pair step, a 16-point FFT in registers, a
//                  radix-8 stage through the wavefront's LDS slice), add the
//                  real-space components (step 8) to their 32 pixels and
//                  store them.
#include <atomic>

#include "gfc_device.hpp"
#include "gfc_launch.hpp"

namespace gfc {

namespace w256 {
constexpr int W = 256;
constexpr int NC = W / 2;           // packed columns
constexpr int D = 8;                // column decimation: lane (c, h) takes rows k_y = 8m + h
constexpr int M = W / D;            // bins per lane in the column phase
constexpr int BLOCK = NC * D;       // 1,024 threads
constexpr int NWAVE = BLOCK / 64;
constexpr int HROWS = W / 2;        // rows per half of the stamp
// LDS has 32 banks of 4 bytes and serves a 64-bit access 16 lanes at a time:
// the 16 lanes are conflict-free when their float2 addresses differ mod 16.
// Row stride of a half, TS = 2 (mod 16): lanes (column c', h) write rows
// 8k + h, addresses 2 h + c' (mod 16); lanes (row y', r) of the row phase
// read columns 8 m + r (and 128 - 8 m - r): 2 y' +- r.
constexpr int TS = 130;
// Slots of the wavefront-private exchanges: entry (i, j) of slot s at
// s * S + 9 i + j.  Column combine (slot = column c', j = h), S = 8 (mod 16):
// writes 8 c' + h, reads 8 c' + 9 h.  Row stage (slot = row y', j = r),
// S = 2 (mod 16): writes 2 y' + r, reads 2 y' + 9 r.
constexpr int CXS = 72;
constexpr int RXS = 82;
// Row stride of the combine twiddle table (float2): odd, so rows h start in
// distinct banks.
constexpr int TWC = 33;
constexpr int LDS_F2 = HROWS * TS;  // 133 KB
static_assert(NWAVE * 8 * CXS <= LDS_F2, "the column exchange slices lie in the half buffer");
static_assert(8 * RXS <= 8 * TS && (8 * TS) % 16 == 0, "a row exchange slice lies in its wavefront's rows");
}  // namespace w256

// Orders a wavefront's LDS accesses across this point (they execute in
// order on the hardware; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v2f* GlobalF2;

__device__ __forceinline__ float2 ld2(GlobalF2 a, int i) {
  const v2f v = a[i];
  return make_float2(v.x, v.y);
}

// Inputs of stamp g that the kernel reads per stamp, as 32-bit words:
// x, y, flux, r_e, e1, e2, mixture id, PSF id (PT), PSF position (EIG).
constexpr int kInWords = 10;

template <bool EIG, bool PT>
__device__ __forceinline__ uint32_t stamp_word(const RenderArgs& p, int64_t g, int i) {
  const float* f = p.x;
  f = i == 1 ? p.y : f;
  f = i == 2 ? p.flux : f;
  f = i == 3 ? p.r_e : f;
  f = i == 4 ? p.e1 : f;
  f = i == 5 ? p.e2 : f;
  if constexpr (EIG) {
    f = i == 8 ? p.psf_px : f;
    f = i == 9 ? p.psf_py : f;
  }
  const int* n = i == 6 ? p.mix_id : nullptr;
  if constexpr (PT) n = i == 7 ? p.psf_id : n;
  const bool word_of_f = i < 6 || (EIG && i >= 8);
  if (word_of_f) return __builtin_bit_cast(uint32_t, f[g]);
  return n ? (uint32_t)n[g] : 0u;
}

// A stamp's galaxy (Step 3) and the bound of its skip test, as 16 words in
// LDS: the first wavefront forms them once and every wavefront reads them.
constexpr int kGalWords = 16;

// From the stamp's input words, word i held by lane i of the wavefront.
template <int W>
__device__ __forceinline__ void publish_galaxy(const RenderArgs& p, uint32_t word, int lane, uint32_t* s_gal) {
  uint32_t w[7];
  static_for<0, 7>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    w[i] = (uint32_t)__builtin_amdgcn_readlane((int)word, i);
  });
  const Galaxy G = make_galaxy<W>(p, GalaxyIn{__builtin_bit_cast(float, w[0]), __builtin_bit_cast(float, w[1]),
                                              __builtin_bit_cast(float, w[2]), __builtin_bit_cast(float, w[3]),
                                              __builtin_bit_cast(float, w[4]), __builtin_bit_cast(float, w[5]),
                                              (int)w[6]});
  const float lamq = -kQ * shape_min_eig(G);
  if (lane == 0) {
    uint4* d = reinterpret_cast<uint4*>(s_gal);
    d[0] = make_uint4(__builtin_bit_cast(uint32_t, G.x0), __builtin_bit_cast(uint32_t, G.y0),
                      __builtin_bit_cast(uint32_t, G.flux), __builtin_bit_cast(uint32_t, G.fx));
    d[1] = make_uint4(__builtin_bit_cast(uint32_t, G.fy), (uint32_t)G.nx, (uint32_t)G.ny,
                      __builtin_bit_cast(uint32_t, G.b11));
    d[2] = make_uint4(__builtin_bit_cast(uint32_t, G.b12), __builtin_bit_cast(uint32_t, G.b22), (uint32_t)G.table,
                      (uint32_t)G.K);
    d[3] = make_uint4(G.ok ? 1u : 0u, __builtin_bit_cast(uint32_t, lamq), 0u, 0u);
  }
}

// The published galaxy, in scalar registers.
__device__ __forceinline__ Galaxy read_galaxy(const uint32_t* s_gal, float* lamq) {
  const uint4* d = reinterpret_cast<const uint4*>(s_gal);
  const uint4 a = d[0], b = d[1], c = d[2], e = d[3];
  auto u = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
  auto f = [&](uint32_t v) { return __builtin_bit_cast(float, u(v)); };
  Galaxy G;
  G.x0 = f(a.x);
  G.y0 = f(a.y);
  G.flux = f(a.z);
  G.fx = f(a.w);
  G.fy = f(b.x);
  G.nx = (int)u(b.y);
  G.ny = (int)u(b.z);
  G.b11 = f(b.w);
  G.b12 = f(c.x);
  G.b22 = f(c.y);
  G.table = (int)u(c.z);
  G.K = (int)u(c.w);
  G.ok = u(e.x) != 0u;
  *lamq = f(e.y);
  return G;
}

// EIG: spatially varying PSF (eigen-PSF components with polynomial weights).
// PT: each galaxy names its constant PSF in p.psf_id (serving batches).
//
// Persistent: the resident workgroups (one per CU: the LDS holds one half of
// a stamp) take stamps in turn.  Lanes 0..9 of the first wavefront load the
// inputs of a workgroup's next stamp while it renders the current one, so a
// stamp starts without a memory round trip, and the first wavefront forms
// the next stamp's galaxy for all sixteen.
template <bool EIG, bool PT>
__global__ void __launch_bounds__(w256::BLOCK) render_w256_kernel(RenderArgs pa) {
  using namespace w256;
  __shared__ float2 s_buf[LDS_F2];
  __shared__ float2 s_py[W + 2];
  __shared__ float2 s_nyq[W];
  __shared__ float s_tw[NC];        // the Nyquist row's omega = -1/2 twin, per column
  __shared__ float4 s_rc[kKmax];    // real-space components: amplitude, g, sxy / syy, -log2(e) / (2 syy)
  // Combine twiddles s_twc[h][8 k + g] = w^(g (8 k + h)), w = exp(2 pi i /
  // 256), rows TWC apart so that a 16-lane group's reads fall in distinct
  // banks.
  __shared__ float2 s_twc[8 * TWC];
  __shared__ float s_cj[kEigMax];   // eigen-PSF component weights at this galaxy's position
  __shared__ uint32_t s_in[kInWords];
  __shared__ __attribute__((aligned(16))) uint32_t s_gal[kGalWords];

  {
    const uint32_t w0 = threadIdx.x < kInWords ? stamp_word<EIG, PT>(pa, blockIdx.x, threadIdx.x) : 0u;
    if (threadIdx.x < kInWords) s_in[threadIdx.x] = w0;
    if (threadIdx.x < 64) publish_galaxy<W>(pa, w0, (int)threadIdx.x, s_gal);
  }
  if (threadIdx.x < 256) {
    const int hh = threadIdx.x >> 5, kg = threadIdx.x & 31;  // kg = 8 k + g
    s_twc[hh * TWC + kg] = twiddle_rt<+1, W>((kg & 7) * (8 * (kg >> 3) + hh));
  }
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront index (scalar)
  for (int64_t stamp = blockIdx.x; stamp < pa.n; stamp += gridDim.x) {
  const RenderArgs& p = kernel_args_renewed<RenderArgs>();
  // The lane index is recomputed per stamp (no vector register is held
  // across stamps); the asm keeps the compiler from hoisting it.
  int lane;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane));
  const int t = wv * 64 + lane;
  __syncthreads();  // s_in holds this stamp's inputs; the previous stamp is done with LDS
  uint32_t in[kInWords];
  static_for<7, kInWords>([&](auto ii) {  // the PSF id (PT) and the PSF position (EIG)
    constexpr int i = decltype(ii)::value;
    in[i] = __builtin_amdgcn_readfirstlane(s_in[i]);
  });
  float lamq_pub;
  Galaxy G = read_galaxy(s_gal, &lamq_pub);
  // PSF spectra are global memory (the pointer read from the PSF table would
  // otherwise be generic and its loads flat, which also count as LDS waits)
  GlobalF2 psfm = (GlobalF2)p.psf_main;
  GlobalF2 psfn = (GlobalF2)p.psf_nyq;
  int ps = 0;
  if constexpr (PT) {
    static_assert(!EIG, "a per-galaxy PSF index takes constant PSFs");
    ps = (int)in[7];
    if (ps < 0 || ps >= p.n_psf) {  // invalid galaxy: NaN stamp, counted
      ps = 0;
      G.ok = false;
      G.flux = __builtin_nanf("");
    }
    psfm = (GlobalF2)p.psf_main_tab[ps];
    psfn = (GlobalF2)p.psf_nyq_tab[ps];
  }
  const float trB = G.b11 + G.b22;
  const float fs = G.flux * (1.f / ((float)W * (float)W));

  // PSF Gaussian (step 2; for a varying PSF from the weighted components' moments)
  float pg[6];
  if constexpr (EIG) {
    const float u = uniform_f((__builtin_bit_cast(float, in[8]) - p.eig_norm[0]) * p.eig_norm[1]);
    const float v = uniform_f((__builtin_bit_cast(float, in[9]) - p.eig_norm[2]) * p.eig_norm[3]);
    const float up[4] = {1.f, u, u * u, u * u * u}, vp[4] = {1.f, v, v * v, v * v * v};
    if (t < p.eig_J) s_cj[t] = eigen_weight(p, t, up, vp);
    __syncthreads();
    float mom[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < p.eig_J; ++j) {
      const float cj = s_cj[j];
      static_for<0, 6>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        mom[i] = fmaf(cj, p.eig_mom[j * 6 + i], mom[i]);
      });
    }
    eigen_gauss(mom, pg);
    static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = uniform_f(pg[decltype(ii)::value]); });
  } else if constexpr (PT) {
    static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg_tab[6 * ps + decltype(ii)::value]; });
  } else {
    static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg[decltype(ii)::value]; });
  }

  // ------------------------------------------------------------ column phase
  const int c = t >> 3, h = t & 7;
  const float nu = (float)c * (1.f / W);
  const float hW = (float)h * (1.f / W);
  const float g0 = kQ * G.b11 * nu * nu;
  const float g1 = 2.f * kQ * G.b12 * nu;
  const float g2 = kQ * G.b22;
  // omega = c_m + h/W with a compile-time c_m: the quadratic expanded about
  // h/W is two FMAs with an immediate per bin
  const float e0 = fmaf(hW, fmaf(g2, hW, g1), g0);
  const float e1 = fmaf(2.f * g2, hW, g1);
  float qv[M];
  static_for<0, M>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    if constexpr (D * m == W / 2) {  // k_y = 128 + h: the Nyquist row (+1/2) for h = 0
      const float om = h ? -0.5f + hW : 0.5f;
      qv[m] = fmaf(om, fmaf(g2, om, g1), g0);
    } else if constexpr (m == 0) {
      qv[m] = e0;
    } else {
      constexpr float cm = (D * m < W / 2) ? (float)(D * m) * (1.f / W) : (float)(D * m - W) * (1.f / W);
      qv[m] = fmaf(cm, fmaf(cm, g2, e1), e0);
    }
  });

  // Threads t < W also take row t of column k_x = W/2: (+-1/2, omN).  The
  // corner's omega = -1/2 twins equal the (-+1/2, +1/2) pair of row W/2
  // (the mixture transform is even).  Threads t < NC take the omega = -1/2
  // twin of the Nyquist row in column t.  Waves 0..3 and 0..1: uniform
  // branches.
  const bool nyq = t < W, twin = t < NC;
  const float omN = (t < W / 2) ? (float)t * (1.f / W) : (t == W / 2 ? 0.5f : (float)(t - W) * (1.f / W));
  float qn[3] = {0.f, 0.f, 0.f};
  if (nyq) {
    const float qa = kQ * G.b11 * 0.25f, qb = kQ * G.b12, qd = kQ * G.b22;
    qn[0] = fmaf(omN, fmaf(qd, omN, qb), qa);
    qn[1] = fmaf(omN, fmaf(qd, omN, -qb), qa);
    const float nt = (float)t * (1.f / W);  // (nt, -1/2)
    qn[2] = kQ * fmaf(nt, fmaf(G.b11, nt, -G.b12), 0.25f * G.b22);
  }

  // Skipping negligible bins: over block b of eight bins (k_y in
  // [64 b, 64 b + 63]) and this wavefront's columns, nu^2 + omega^2 >= r2[b],
  // so a component's exponent is at most -v lamq r2[b].
  const float lamq = lamq_pub;
  int wvs = wv;  // renewed per stamp: the bounds below are not held across stamps
  asm volatile("" : "+s"(wvs));
  const float nlo = (float)(8 * wvs) * (1.f / W);
  // A component of variance v is evaluated in block b when v < vmax[b]
  // (vmax = +inf when lambda or the radius is zero).
  const float r2[4] = {nlo * nlo, fmaf(nlo, nlo, 0.0625f), fmaf(nlo, nlo, (65.f * 65.f) / (256.f * 256.f)),
                       fmaf(nlo, nlo, 1.f / (256.f * 256.f))};
  float vmax[4];
  static_for<0, 4>([&](auto bb) {
    constexpr int b = decltype(bb)::value;
    vmax[b] = uniform_f(kSkipLog2 * __builtin_amdgcn_rcpf(lamq * r2[b]));  // rcp(0) = +inf
  });
  const float vmaxN = uniform_f(kSkipLog2 * __builtin_amdgcn_rcpf(lamq * 0.25f));  // |nu| = 1/2 or |omega| = 1/2
  float S[M];
  float SN[3] = {0.f, 0.f, 0.f};
  static_for<0, M>([&](auto mm) { S[decltype(mm)::value] = 0.f; });
  // Lane k of every wavefront works out component k's route weight (K <= 16
  // lanes), the loop takes v and w A from it by lane reads, and lane k of
  // the first wavefront forms the component's real-space constants.
  float vk = 0.f, wak = 0.f;
  bool rk = false;
  {
    const int lk = lane;
    if (lk < G.K) {
      vk = p.var[G.table * kKmax + lk];
      const float Ak = p.amp[G.table * kKmax + lk];
      const float wk = route_weight<W>(vk * trB, p.flags);
      wak = wk * Ak;
      rk = wk < 1.f && Ak != 0.f;
      if (rk && t == lk) {
        // the component convolved with the PSF Gaussian: covariance
        // v B + C_p, amplitude (1 - w) A flux a_p / (2 pi sqrt(det))
        const float sxx = fmaf(vk, G.b11, pg[2]);
        const float sxy = fmaf(vk, G.b12, pg[3]);
        const float syy = fmaf(vk, G.b22, pg[4]);
        const float det = fmaf(sxx, syy, -(sxy * sxy));
        const float rsyy = __builtin_amdgcn_rcpf(syy);
        s_rc[lk] = make_float4((1.f - wk) * Ak * G.flux * pg[5] * kInv2Pi * __builtin_amdgcn_rsqf(det),
                               __builtin_amdgcn_sqrtf(-kHalfLog2e * syy * __builtin_amdgcn_rcpf(det)), sxy * rsyy,
                               kHalfLog2e * rsyy);
      }
    }
  }
  const unsigned rmask = (unsigned)__ballot(rk) & ((1u << kKmax) - 1u);
  for (int k = 0; k < G.K; ++k) {
    const float wa = lane_f(wak, k);
    if (wa == 0.f) continue;
    const float v = lane_f(vk, k);
    static_for<0, M / 8>([&](auto bb) {
      constexpr int b = decltype(bb)::value;
      if (v < vmax[b]) {
        static_for<0, 8>([&](auto ii) {
          constexpr int m = 8 * b + decltype(ii)::value;
          S[m] = fmaf(wa, __builtin_amdgcn_exp2f(v * qv[m]), S[m]);
        });
      }
    });
    if (nyq && v < vmaxN) {
      SN[0] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[0]), SN[0]);
      SN[1] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[1]), SN[1]);
      if (twin) SN[2] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[2]), SN[2]);
    }
  }

  // y phases (shift theorem, with the integer part of y as an exact table
  // entry) and the Nyquist column, row t
  if (nyq) {
    float sy, cy, sxh, cxh;
    sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
    {
      const float2 ti = twiddle_rt<-1, W>(G.ny * t);
      const float c2 = fmaf(cy, ti.x, -(sy * ti.y)), s2 = fmaf(cy, ti.y, sy * ti.x);
      cy = c2;
      sy = s2;
    }
    sincospi_poly(-G.fx, &sxh, &cxh);
    s_py[t] = make_float2(cy, sy);
    if (twin) s_tw[t] = SN[2];
    if (t == W / 2) s_py[W] = make_float2(cy, -sy);  // omega = -1/2 (the integer part's phase is real there)
    float2 psfN;
    if constexpr (EIG) {
      psfN = make_float2(0.f, 0.f);
      for (int j = 0; j < p.eig_J; ++j) {
        const float cj = s_cj[j];
        const float2 q = p.psf_nyq[j * p.eig_stride + t];
        psfN = make_float2(fmaf(cj, q.x, psfN.x), fmaf(cj, q.y, psfN.y));
      }
    } else {
      psfN = ld2(psfn, t);
    }
    const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
    const bool corner = (t == W / 2);
    const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
    const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
    const float2 plus = cadd(cscale(pyA, SN[0]), cscale(pyB, SN[1]));
    const float2 minus = cadd(cscale(pyA, SN[1]), cscale(pyB, SN[0]));
    // the integer x shift at k_x = W/2 is exp(-i pi n_x) = +-1
    const float sgn = (G.nx & 1) ? -1.f : 1.f;
    s_nyq[t] = cmul(cscale(psfN, 0.5f * fs * sgn), cadd(cmul(eM, plus), cmul(eP, minus)));
  }
  __syncthreads();

  // x phase of column c (fractional part by polynomial, integer part exact)
  float2 pxF;
  {
    float sx, cx;
    sincospi_poly(-2.f * G.fx * nu, &sx, &cx);
    const float2 tx = twiddle_rt<-1, W>(G.nx * c);
    pxF = cscale(cmul(make_float2(cx, sx), tx), fs);
  }
  // Cached PSF spectrum in the decimation-4 lane order: bin (k_y, c) at
  // (k_y / 4) (4 NC) + 4 c + k_y mod 4, with k_y = 8 m + h.  Eight bins at a
  // time (for a varying PSF the component loop runs inside each group).
  float2 Z[M];
  const int pidx0 = (h >> 2) * (4 * NC) + 4 * c + (h & 3);
  static_for<0, M / 8>([&](auto gg) {
    constexpr int g = decltype(gg)::value;
    float2 P[8];
    if constexpr (EIG) {
      static_for<0, 8>([&](auto ii) { P[decltype(ii)::value] = make_float2(0.f, 0.f); });
#pragma unroll 1
      for (int j = 0; j < p.eig_J; ++j) {
        const float cj = s_cj[j];
        const float2* q = p.psf_main + (int64_t)j * p.eig_stride + pidx0;
        static_for<0, 8>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          const float2 v = q[2 * (8 * g + i) * (4 * NC)];
          P[i] = make_float2(fmaf(cj, v.x, P[i].x), fmaf(cj, v.y, P[i].y));
        });
      }
    }
    static_for<0, 8>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int m = 8 * g + i;
      if constexpr (!EIG) P[i] = ld2(psfm, pidx0 + 2 * m * (4 * NC));
      if constexpr (D * m == W / 2) {
        const float2 q0 = s_py[W / 2 + h];
        const float2 pyA = h ? q0 : cscale(q0, 0.5f);
        const float2 pyB = h ? make_float2(0.f, 0.f) : cscale(s_py[W], 0.5f);
        Z[m] = cmul(cmul(P[i], pxF), cadd(cscale(pyA, S[m]), cscale(pyB, s_tw[c])));
      } else {
        Z[m] = cscale(cmul(cmul(P[i], s_py[D * m + h]), pxF), S[m]);
      }
    });
    __builtin_amdgcn_sched_barrier(0);  // bounds the PSF loads in flight
  });
  if (c == 0) {  // column 0 carries column W/2 as its imaginary part
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 xn = s_nyq[D * m + h];
      Z[m] = make_float2(Z[m].x - xn.y, Z[m].y + xn.x);
    });
  }
  fft<M, +1>(Z);  // Z[j] = E_h[j] = sum_m X[8m + h] exp(2 pi i m j / 32)

  // ------------------------------------------------------------ column combine
  // x[c][j + 32 q] = sum_g exp(2 pi i g q / 8) (exp(2 pi i g j / 256) E_g[j]):
  // chunk k hands E_h[8k .. 8k + 7] over so that lane h gets E_0..7[8k + h].
  float2 X4[4][8];
  {
    float2* cxb = s_buf + wv * (8 * CXS) + (lane >> 3) * CXS;  // this column's slot
    static_for<0, 4>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      __builtin_amdgcn_sched_barrier(0);  // one chunk's twiddle loads in flight at a time
      static_for<0, 8>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        cxb[9 * i + h] = Z[8 * k + i];
      });
      wave_lds_sync();
      float2 a[8];
      static_for<0, 8>([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        a[g] = cxb[9 * h + g];
      });
      wave_lds_sync();  // read before the next chunk overwrites the slot
      // w^(g j), j = 8 k + h
      const float2* tw = s_twc + h * TWC + 8 * k;
      static_for<1, 8>([&](auto gg) {
        constexpr int g = decltype(gg)::value;
        a[g] = cmul(a[g], tw[g]);
      });
      fft<8, +1>(a);
      static_for<0, 8>([&](auto qq) { X4[k][decltype(qq)::value] = a[decltype(qq)::value]; });
    });
  }

  // ------------------------------------------------------------ row phase, per half
  float* outp = p.out + stamp * (int64_t)(W * W);
  uint32_t in_next = 0;
  static_for<0, 2>([&](auto hh) {
    constexpr int half = decltype(hh)::value;
    // Row-phase lane: row 8 wv + yl of the half, class r.  The lane index is
    // renewed opaquely per half, so the twiddles and addresses derived from
    // it are recomputed instead of being held in registers across the half.
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int yl = ln & 7, r = ln >> 3;
    __syncthreads();  // the previous users of s_buf are done
    // rows 8k + h + 32 qq of the half (q = 4 half + qq), column c
    static_for<0, 4>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      static_for<0, 4>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        s_buf[(8 * k + h + 32 * q) * TS + c] = X4[k][4 * half + q];
      });
    });
    __syncthreads();
    if constexpr (half == 1) {
      // the next stamp's inputs, in flight while this half is finished
      const int64_t next = stamp + gridDim.x;
      if (t < kInWords && next < p.n) in_next = stamp_word<EIG, PT>(p, next, t);
    }
    const int yloc = 8 * wv + yl;
    const int y = half * HROWS + yloc;
    // pair step: R[m] for k_x = 8m + r, from X[k] and X[128 - k] of this row
    float2 R[16];
    {
      const float2* row = s_buf + yloc * TS;
      const float2 wr = s_twc[r * TWC + 1];  // w^r
      static_for<0, 16>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const int k = 8 * m + r;
        float2 a = row[k];
        float2 b = row[(NC - k) & (NC - 1)];
        if (m == 0 && r == 0) {  // packed column 0: X[0] = real part, X[128] = imaginary part
          b = make_float2(a.y, 0.f);
          a = make_float2(a.x, 0.f);
        } else {
          b = cconj(b);
        }
        // s + i w^k (a - b), w = exp(2 pi i / 256): w^k = w^r exp(2 pi i m / 32),
        // the second factor as a compile-time scale times two FMAs
        using T = TwFactor<+1, 32, m>;
        const float2 s = cadd(a, b);
        const float2 u = T::unit(cmul(wr, csub(a, b)));
        R[m] = make_float2(fmaf(-T::r, u.y, s.x), fmaf(T::r, u.x, s.y));
      });
    }
    fft<16, +1>(R);   // R[n1] = sum_m R_in[m] exp(2 pi i m n1 / 16)
    static_for<1, 16>([&](auto nn) {
      constexpr int n1 = decltype(nn)::value;
      R[n1] = cmul(R[n1], twiddle_rt<+1, 128>(r * n1));
    });
    // z[n1 + 16 q] = sum_r exp(2 pi i r q / 8) R_r[n1]: chunk kk hands the
    // classes' R_r[n1] for n1 = kk (mod 2) over so that lane r gets
    // R_0..7[2 r + kk]
    float2 zq[2][8];
    {
      // This wavefront's slice lies in the eight rows of the half that only
      // it reads (rows 8 wv .. 8 wv + 7, read above): no barrier is needed
      // before it is reused.
      float2* rxb = s_buf + wv * (8 * TS) + yl * RXS;  // this row's slot
      static_for<0, 2>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        static_for<0, 8>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          rxb[9 * i + r] = R[2 * i + k];
        });
        wave_lds_sync();
        float2 a[8];
        static_for<0, 8>([&](auto gg) {
          constexpr int g = decltype(gg)::value;
          a[g] = rxb[9 * r + g];
        });
        wave_lds_sync();
        fft<8, +1>(a);
        static_for<0, 8>([&](auto qq) { zq[k][decltype(qq)::value] = a[decltype(qq)::value]; });
      });
    }
    // z[n] = I[2n] + i I[2n + 1] with n = 2 r + kk + 16 q: lane r holds
    // pixels x = 4 r + 32 q + 0..3 (zq[0][q], then zq[1][q])
    if (rmask != 0) {
      const float dy = (float)y - G.y0 - pg[1];
      const float dx0 = -G.x0 - pg[0];  // dx of column 0
      for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
        const float4 rc = s_rc[__builtin_ctz(mk)];
        const float ampr = rc.x, g = rc.y;
        // along the row (dy fixed) the quadratic form is dy^2 / syy +
        // (syy / det) (dx - (sxy / syy) dy)^2, completed about the conditional
        // mean: with dx = x + dx0 the exponent is k - u^2, u = g (x + m)
        const float k0 = rc.w * dy * dy;
        const float gm = g * fmaf(-rc.z, dy, dx0 + (float)(4 * r));  // x measured from this lane's 4 r
        static_for<0, 8>([&](auto qq) {
          constexpr int q = decltype(qq)::value;
          constexpr float xo = (float)(32 * q);
          const float u0 = fmaf(g, xo, gm), u1 = fmaf(g, xo + 1.f, gm);
          const float u2 = fmaf(g, xo + 2.f, gm), u3 = fmaf(g, xo + 3.f, gm);
          zq[0][q].x = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u0, u0, k0)), zq[0][q].x);
          zq[0][q].y = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u1, u1, k0)), zq[0][q].y);
          zq[1][q].x = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u2, u2, k0)), zq[1][q].x);
          zq[1][q].y = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u3, u3, k0)), zq[1][q].y);
        });
      }
    }
    // eight lanes store one 128-byte segment of the row
    float* orow = outp + (int64_t)y * W + 4 * r;
    const bool acc = (p.flags & kAccumulate) != 0;
    static_for<0, 8>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      v4f* dst = reinterpret_cast<v4f*>(orow + 32 * q);
      v4f val = {zq[0][q].x, zq[0][q].y, zq[1][q].x, zq[1][q].y};
      if (acc) val += *dst;
      __builtin_nontemporal_store(val, dst);
    });
  });
  if (!G.ok && t == 0) atomicAdd(p.invalid, 1ull);
  // every thread read s_in and s_gal at this stamp's start, before the
  // barriers above
  if (t < kInWords) s_in[t] = in_next;
  if (wv == 0) publish_galaxy<W>(p, in_next, lane, s_gal);
  }  // stamps of this workgroup
}

// Workgroups of one instantiation resident at once on the current device
// (one per CU), queried once per device.
// (Launches from several host threads may fill an entry at once; they store
// the same value.)
template <bool EIG, bool PT>
static hipError_t w256_resident(int64_t* out) {
  constexpr int kMaxDev = 64;
  static std::atomic<int64_t> cached[kMaxDev];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  int64_t v = cached[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cus = 0, per = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, render_w256_kernel<EIG, PT>, w256::BLOCK, 0);
    if (e != hipSuccess) return e;
    v = (int64_t)std::max(per, 1) * std::max(cus, 1);
    cached[dev].store(v, std::memory_order_relaxed);
  }
  *out = v;
  return hipSuccess;
}

template <bool EIG, bool PT>
static hipError_t launch_w256(const RenderArgs& args, hipStream_t stream) {
  if (args.n <= 0) return hipSuccess;
  int64_t resident = 0;
  hipError_t e = w256_resident<EIG, PT>(&resident);
  if (e != hipSuccess) return e;
  const int64_t nb = std::min<int64_t>(args.n, resident);
  hipLaunchKernelGGL((render_w256_kernel<EIG, PT>), dim3((unsigned)nb), dim3(w256::BLOCK), 0, stream, args);
  return hipGetLastError();
}

hipError_t launch_render_w256(const RenderArgs& args, hipStream_t stream) {
  if (args.psf_id) return args.eig_J > 0 ? hipErrorInvalidValue : launch_w256<false, true>(args, stream);
  return args.eig_J > 0 ? launch_w256<true, false>(args, stream) : launch_w256<false, false>(args, stream);
}

}  // namespace gfc
