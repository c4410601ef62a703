// Forward render kernel for stamp sizes W = 16, 32, 64, 128 (Lang 2020,
// Section 2, steps 3-8), one fused kernel per launch.
//
// A stamp is handled by W lanes (W < 64: 64/W stamps per wavefront; W = 128:
// two wavefronts).  The half spectrum (W/2 + 1 columns) never leaves the chip:
//
//  column phase  lane (c, h), c = 0..W/2-1, h = 0..1, owns column k_x = c and
//                rows k_y = 2m + h.  It evaluates the mixture transform
//                (steps 5-6) on those bins, multiplies by the fractional-shift
//                phase, the flux and the cached PSF spectrum (step 7a), and
//                runs a W/2-point inverse FFT in registers (the even/odd half
//                of the length-W column transform).  Column k_x = W/2 is
//                packed into column 0 as its imaginary part: both columns
//                transform to real vectors because the product is Hermitian.
//  transpose     through LDS; the last radix-2 stage of the column transform
//                is applied while reading back.
//  row phase     lane y owns row y and runs the length-W complex-to-real
//                inverse transform as a W/2-point complex FFT in registers.
//  store         rows go through LDS with the integer part of the x centre
//                applied as a cyclic roll (the integer part of y is a phase
//                in the y-phase table), then real-space components (step 8)
//                are added and stamps are written coalesced.
#include "gfc_device.hpp"
#include "gfc_launch.hpp"

namespace gfc {

template <int W, bool EIG = false>
struct SmallCfg {
  static constexpr int M = W / 2;                // values per lane in the column phase
  // With a varying PSF at 64 x 64, four stamps (one per wavefront) share a
  // workgroup and stream each component spectrum through LDS once for all four.
  static constexpr bool SHARE = EIG && W == 64;
  static constexpr int BLOCK = SHARE ? 256 : (W < 64 ? 64 : W);  // threads per workgroup
  static constexpr int SPB = BLOCK / W;          // stamps per workgroup
  static constexpr bool WAVE1 = W >= 64;         // one stamp per wavefront (or two wavefronts per stamp)
  // Both LDS transposes run in two passes over halves of the data, so a
  // stamp needs half the LDS and more wavefronts fit on a CU.
  static constexpr int T1S = W / 2 + 1;          // float2 per row: W/4 columns x 2 halves + pad
  static constexpr int T1N = M * T1S;            // float2 per stamp; also (W/2) x (W+1) floats
  static constexpr int HR = W / 2;               // rows of the store tile per pass
};

// EIG: the PSF varies over the image (eigen-PSF components with polynomial
// weights); its spectrum and Gaussian are formed per stamp from the
// components' cached spectra and moments.
// W = 128 is held to two wavefronts per SIMD (a small spill costs less than
// running one wavefront per SIMD); the other sizes reach their occupancy freely.
// LZ (W <= 64): the Lanczos-3 sub-pixel shift is applied while storing.
// PT: each galaxy names its (constant) PSF in p.psf_id, and the stamp takes
// that PSF's spectrum and Gaussian from the tables (a serving batch mixes
// PSFs); the one-PSF instantiations compile exactly as without it.
template <int W, bool EIG, bool LZ, bool PT>
__global__ void __launch_bounds__((SmallCfg<W, EIG>::BLOCK)) __attribute__((amdgpu_waves_per_eu(W == 128 ? 2 : 1)))
render_small_kernel(RenderArgs p) {
  using C = SmallCfg<W, EIG>;
  constexpr int M = C::M;
  constexpr int T1S = C::T1S;
  __shared__ __attribute__((aligned(16))) float2 s_t1[C::SPB][C::T1N];  // 16-byte aligned: also read as float4
  __shared__ float2 s_py[C::SPB][W + 2];
  __shared__ float2 s_nyq[C::SPB][W];
  __shared__ float2 s_rs[C::SPB][kKmax];  // (v, (1 - w) A) of the components with a real-space share
  // per real-space component, its column constants (g, amplitude, -sxy / sxx,
  // log2(e) / (2 sxx)) of the store below (not with the fused Lanczos shift)
  __shared__ float4 s_rc[C::SPB][LZ ? 1 : kKmax];
  __shared__ float s_lw[C::SPB][12];      // raw Lanczos weights of the stamp (fused shift, W <= 64)

  const int l = (C::SPB == 1) ? (int)threadIdx.x : (int)threadIdx.x % W;
  int slot = (C::SPB == 1) ? 0 : (int)threadIdx.x / W;
  if constexpr (C::WAVE1 && C::SPB > 1) slot = __builtin_amdgcn_readfirstlane(slot);  // keeps the stamp index scalar
  const int64_t stamp = (int64_t)blockIdx.x * C::SPB + slot;
  const bool live = stamp < p.n;
  Galaxy G = load_galaxy<W>(p, live ? stamp : p.n - 1);
  if constexpr (C::WAVE1) {  // one stamp per wavefront: keep its integer shift in SGPRs
    make_uniform(G);
  }
  // This stamp's PSF spectrum (lane-permuted main columns, Nyquist column)
  // and the index of its Gaussian in the table (PT).
  const float2* psfm = p.psf_main;
  const float2* psfn = p.psf_nyq;
  int ps = 0;
  if constexpr (PT) {
    static_assert(!EIG, "a per-galaxy PSF index takes constant PSFs");
    ps = p.psf_id[live ? stamp : p.n - 1];
    if constexpr (C::WAVE1) ps = __builtin_amdgcn_readfirstlane(ps);
    if (ps < 0 || ps >= p.n_psf) {  // invalid galaxy: NaN stamp, counted
      ps = 0;
      G.ok = false;
      G.flux = __builtin_nanf("");
    }
    psfm = p.psf_main_tab[ps];
    psfn = p.psf_nyq_tab[ps];
  }
  // Lanczos-3 weights of the fused shift (taps d = -3..2 along x, then y),
  // formed up front: with one stamp per wavefront they sit in scalar
  // registers until the store.
  float wxn[6], wy[6];
  if constexpr (LZ) {
    const int64_t gs = live ? stamp : p.n - 1;
    if (l < 12) {  // raw weights of taps d = -3..2: x in 0..5, y in 6..11
      const float v = l < 6 ? p.x[gs] : p.y[gs];
      s_lw[slot][l] = lanczos3((float)((l % 6) - 3) + (v - floorf(v)));
    }
    float wx[6], sx = 0.f, sy = 0.f;  // (one wavefront per slot: no barrier needed)
    static_for<0, 6>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      wx[d] = s_lw[slot][d];
      wy[d] = s_lw[slot][6 + d];
      sx += wx[d];
      sy += wy[d];
    });
    const float rx = 1.f / sx, ry = 1.f / sy;
    static_for<0, 6>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      wxn[d] = wx[d] * rx;
      wy[d] *= ry;
      if constexpr (C::WAVE1) {  // one stamp per wavefront: the weights are uniform
        wxn[d] = uniform_f(wxn[d]);
        wy[d] = uniform_f(wy[d]);
      }
    });
  }
  if constexpr (LZ) {
    // The galaxy sits at its integer position (the fractional part is the
    // Lanczos shift), and that integer shift is applied as a Fourier phase as
    // well (cyclic shift theorem) instead of a roll at the store: the stamp
    // then leaves the row transform in output order, so the filter's edges
    // are fixed at compile time.
    G.fx = (float)G.nx;
    G.fy = (float)G.ny;
  }
  const float* amp = p.amp + G.table * kKmax;
  const float* var = p.var + G.table * kKmax;
  const int kloop = C::WAVE1 ? G.K : p.kmax;
  const float trB = G.b11 + G.b22;

  // ---------------------------------------------------------------- column phase
  const int c = l >> 1, h = l & 1;
  const float nu = (float)c * (1.f / W);
  const float hW = (float)h * (1.f / W);
  // exponent per unit mixture variance: kQ (b11 nu^2 + 2 b12 nu om + b22 om^2)
  const float g0 = kQ * G.b11 * nu * nu;
  const float g1 = 2.f * kQ * G.b12 * nu;
  const float g2 = kQ * G.b22;
  // Row k_y = 2m + h has omega = c_m + h/W with a compile-time c_m, so the
  // quadratic is expanded about h/W: q = e0 + c_m (e1 + c_m g2), two FMAs
  // with an immediate c_m per bin (e0 = q(h/W), e1 = q'(h/W); for h = 0 they
  // are g0 and g1 and the result is the plain quadratic in omega).
  const float e0 = fmaf(hW, fmaf(g2, hW, g1), g0);
  const float e1 = fmaf(2.f * g2, hW, g1);
  float qv[M + 1];
  static_for<0, M>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    if constexpr (2 * m == W / 2) {
      const float om = h ? (float)(W / 2 + 1 - W) * (1.f / W) : 0.5f;
      qv[m] = fmaf(om, fmaf(g2, om, g1), g0);
    } else if constexpr (m == 0) {
      qv[m] = e0;
    } else {
      constexpr float cm = (2 * m < W / 2) ? (float)(2 * m) * (1.f / W) : (float)(2 * m - W) * (1.f / W);
      qv[m] = fmaf(cm, fmaf(cm, g2, e1), e0);
    }
  });
  // Nyquist column k_x = W/2: lane l takes row k_y = l at nu = +1/2 and -1/2.
  // The corner's omega = -1/2 twins need no evaluation of their own: the
  // mixture transform is even, so (+-1/2, -1/2) equals (-+1/2, +1/2), the
  // pair that lane W/2 (omega = +1/2) holds.  Up to 64 x 64 the -1/2 values
  // need no evaluation either: (-1/2, omega_l) equals (+1/2, -omega_l), lane
  // W - l's, except at the corner, whose (-1/2, +1/2) the h = 1 lanes
  // evaluate in slot M (where the h = 0 lanes hold the Nyquist row's
  // omega = -1/2 twin and the h = 1 lanes would repeat it).
  constexpr bool kMirrorN = W <= 64;
  constexpr int NQ = kMirrorN ? 1 : 2;
  const float omN = (l < W / 2) ? (float)l * (1.f / W) : (l == W / 2 ? 0.5f : (float)(l - W) * (1.f / W));
  const float qa = kQ * G.b11 * 0.25f, qb = kQ * G.b12, qd = kQ * G.b22;
  float qn[2];
  qn[0] = fmaf(omN, fmaf(qd, omN, qb), qa);      // (+1/2, omN)
  qn[1] = fmaf(omN, fmaf(qd, omN, -qb), qa);     // (-1/2, omN)
  qv[M] = fmaf(-0.5f, fmaf(g2, -0.5f, g1), g0);  // Nyquist row, omega = -1/2
  if constexpr (kMirrorN) {
    if (h) qv[M] = fmaf(0.5f, fmaf(qd, 0.5f, -qb), qa);  // the corner (-1/2, +1/2)
  }

  // PSF spectrum of this lane's bins and the PSF Gaussian (step 2; for a
  // varying PSF, the weighted sum of the components at the galaxy's image
  // position, whose transforms and moments are linear in the weights).
  float2 Pm[M];
  float2 psfN;
  float pg[6];
  // With a varying PSF (W <= 64) the components' spectra are summed before
  // the mixture loop, while its sums are not yet live (more registers for
  // the LDS reads in flight); otherwise the spectrum is formed after it.
  constexpr bool kPsfFirst = EIG && W <= 64;
  // At 64 and 128 a constant PSF's spectrum is read in the PSF product
  // itself, 16 bins at a time, rather than all at once while the mixture
  // sums are live: 144 -> 116 VGPRs at 64 (four wavefronts per SIMD instead
  // of three), no spill at 128.
  constexpr bool kPsfStream = !EIG && W >= 64;
  auto psf_terms = [&]() {
    if constexpr (EIG) {
      const int64_t g = live ? stamp : p.n - 1;
      float u = (p.psf_px[g] - p.eig_norm[0]) * p.eig_norm[1];
      float v = (p.psf_py[g] - p.eig_norm[2]) * p.eig_norm[3];
      if constexpr (C::WAVE1) {
        u = uniform_f(u);
        v = uniform_f(v);
      }
      const float up[4] = {1.f, u, u * u, u * u * u}, vp[4] = {1.f, v, v * v, v * v * v};
      float mom[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if constexpr (!C::SHARE) {
        static_for<0, M>([&](auto mm) { Pm[decltype(mm)::value] = make_float2(0.f, 0.f); });
        psfN = make_float2(0.f, 0.f);
      }
      if constexpr (C::SHARE) {
        // Component j (its main bins, then its Nyquist column: contiguous in
        // the cache) is copied into one half of the workgroup's transpose
        // buffers, which are free until the column FFT, while the four
        // wavefronts sum component j - 1 from the other half.  Reading a half
        // again two components later is ordered by the barrier in between.
        constexpr int NS = M * W + W;                   // float2 per component
        constexpr int NV = NS / 2;                      // float4 per component
        constexpr int PER = (NV + C::BLOCK - 1) / C::BLOCK;
        static_assert(2 * NS <= C::SPB * C::T1N, "two component spectra fit in the transpose buffers");
        float2* buf = &s_t1[0][0];
        const float4* src = reinterpret_cast<const float4*>(p.psf_main);
        const int64_t sv = p.eig_stride / 2;  // float4 from one component to the next
        // staged float4 i of this thread: index threadIdx.x + i BLOCK, clamped
        // (the last group is partial; clamped lanes re-read and skip the store)
        float4 st0, st1, st2, st3, st4;
        static_assert(PER == 5, "five float4 per thread at 64 x 64");
        const int i4 = min((int)threadIdx.x + 4 * C::BLOCK, NV - 1);
        const bool w4 = (int)threadIdx.x + 4 * C::BLOCK < NV;
        const float4* s0 = src + threadIdx.x;
        st0 = s0[0]; st1 = s0[C::BLOCK]; st2 = s0[2 * C::BLOCK]; st3 = s0[3 * C::BLOCK]; st4 = src[i4];
        // the component weights, lane k evaluating component k's polynomial
        // (J <= 16 lanes); the loop reads them back with a lane read
        static_assert(C::WAVE1, "one stamp per wavefront");
        const float ck = (l < p.eig_J) ? eigen_weight(p, l, up, vp) : 0.f;
        for (int j = 0; j < p.eig_J; ++j) {
          float4* dst = reinterpret_cast<float4*>(buf + (j & 1) * NS) + threadIdx.x;
          dst[0] = st0; dst[C::BLOCK] = st1; dst[2 * C::BLOCK] = st2; dst[3 * C::BLOCK] = st3;
          if (w4) dst[4 * C::BLOCK] = st4;
          __syncthreads();
          if (j + 1 < p.eig_J) {  // in flight while component j is summed
            const float4* sj = src + (j + 1) * sv;
            st0 = sj[threadIdx.x]; st1 = sj[threadIdx.x + C::BLOCK]; st2 = sj[threadIdx.x + 2 * C::BLOCK];
            st3 = sj[threadIdx.x + 3 * C::BLOCK]; st4 = sj[i4];
          }
          const float cj = lane_f(ck, j);
          const float2* pj = buf + (j & 1) * NS;
          if (j == 0) {  // the first component initialises the sums (eig_J >= 1)
            static_for<0, M>([&](auto mm) {
              constexpr int m = decltype(mm)::value;
              Pm[m] = cscale(pj[m * W + l], cj);
            });
            psfN = cscale(pj[M * W + l], cj);
          } else {
            static_for<0, M>([&](auto mm) {
              constexpr int m = decltype(mm)::value;
              const float2 q = pj[m * W + l];
              Pm[m] = make_float2(fmaf(cj, q.x, Pm[m].x), fmaf(cj, q.y, Pm[m].y));
            });
            const float2 qn = pj[M * W + l];
            psfN = make_float2(fmaf(cj, qn.x, psfN.x), fmaf(cj, qn.y, psfN.y));
          }
          static_for<0, 6>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            mom[i] = fmaf(cj, p.eig_mom[j * 6 + i], mom[i]);
          });
        }
      } else {
        for (int j = 0; j < p.eig_J; ++j) {
          const float cj = eigen_weight(p, j, up, vp);
          const float2* pj = p.psf_main + j * p.eig_stride;
          static_for<0, M>([&](auto mm) {
            constexpr int m = decltype(mm)::value;
            const float2 q = pj[m * W + l];
            Pm[m] = make_float2(fmaf(cj, q.x, Pm[m].x), fmaf(cj, q.y, Pm[m].y));
          });
          const float2 qn = p.psf_nyq[j * p.eig_stride + l];
          psfN = make_float2(fmaf(cj, qn.x, psfN.x), fmaf(cj, qn.y, psfN.y));
          static_for<0, 6>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            mom[i] = fmaf(cj, p.eig_mom[j * 6 + i], mom[i]);
          });
        }
      }
      eigen_gauss(mom, pg);
    } else {
      if constexpr (!kPsfStream) {
        static_for<0, M>([&](auto mm) {
          constexpr int m = decltype(mm)::value;
          Pm[m] = psfm[m * W + l];
        });
      }
      psfN = psfn[l];
      if constexpr (PT) {
        static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg_tab[6 * ps + decltype(ii)::value]; });
      } else {
        static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg[decltype(ii)::value]; });
      }
    }
  };
  if constexpr (kPsfFirst) psf_terms();

  // Component 0 initialises the sums (every table has one; with zero Fourier
  // weight it contributes zeros), the rest accumulate.
  float S[M + 1];
  float SN[2];
  unsigned rmask = 0;  // components with a real-space share
  auto first_terms = [&](float v, float wa) {
    static_for<0, M + 1>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      S[m] = wa * __builtin_amdgcn_exp2f(v * qv[m]);
    });
    static_for<0, NQ>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      SN[j] = wa * __builtin_amdgcn_exp2f(v * qn[j]);
    });
  };
  auto add_terms = [&](float v, float wa) {
    static_for<0, M + 1>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      S[m] = fmaf(wa, __builtin_amdgcn_exp2f(v * qv[m]), S[m]);
    });
    static_for<0, NQ>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      SN[j] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[j]), SN[j]);
    });
  };
  if constexpr (C::WAVE1) {
    // One stamp per wavefront: lane k works out the route weight of component
    // k once (K <= 16 lanes), and the loop takes v and w A from lane k.
    const int lk = (int)__lane_id();
    float vk = 0.f, wak = 0.f;
    bool rk = false;
    if (lk < G.K) {
      vk = var[lk];
      const float Ak = amp[lk];
      const float wk = route_weight<W>(vk * trB, p.flags);
      wak = wk * Ak;
      rk = wk < 1.f && Ak != 0.f;
      if (rk && l == lk) s_rs[slot][lk] = make_float2(vk, (1.f - wk) * Ak);
    }
    rmask = (unsigned)__ballot(rk);
    first_terms(lane_f(vk, 0), lane_f(wak, 0));
    for (int k = 1; k < G.K; ++k) {
      const float wa = lane_f(wak, k);
      if ((__builtin_bit_cast(unsigned, wa) << 1) == 0u) continue;  // w A = +-0
      add_terms(lane_f(vk, k), wa);
    }
  } else {
    // Several stamps per wavefront: lane k of each stamp works out its
    // stamp's component k (K <= W lanes), and the loop takes v and w A from
    // it with a lane permute within the stamp's W lanes.
    float vk = 0.f, wak = 0.f;
    bool rk = false;
    if (l < G.K) {
      vk = var[l];
      const float Ak = amp[l];
      const float wk = route_weight<W>(vk * trB, p.flags);
      wak = wk * Ak;
      rk = wk < 1.f && Ak != 0.f;
      if (rk) s_rs[slot][l] = make_float2(vk, (1.f - wk) * Ak);
    }
    const unsigned long long rb = __ballot(rk);
    rmask = (unsigned)(rb >> ((int)__lane_id() & ~(W - 1))) & (unsigned)((1ull << W) - 1ull);
    first_terms(__shfl(vk, 0, W), __shfl(wak, 0, W));
    for (int k = 1; k < kloop; ++k) {
      const float wa = __shfl(wak, k, W);
      if (wa == 0.f) continue;
      add_terms(__shfl(vk, k, W), wa);
    }
  }

  if constexpr (!kPsfFirst) psf_terms();
  if constexpr (kMirrorN) {
    const float mirrored = __shfl(SN[0], (W - l) & (W - 1), W);
    const float cornerv = __shfl(S[M], 1, W);  // lane 1 of the stamp: h = 1
    SN[1] = (l == W / 2) ? cornerv : mirrored;
  }
  if constexpr (!LZ) {
    // Lane k forms real-space component k's constants once per stamp; they
    // do not depend on the lane's column.
    if (l < kKmax && ((rmask >> l) & 1u)) {
      const float2 rs = s_rs[slot][l];
      const float v = rs.x, ra = rs.y;
      const float sxx = fmaf(v, G.b11, pg[2]);
      const float sxy = fmaf(v, G.b12, pg[3]);
      const float syy = fmaf(v, G.b22, pg[4]);
      const float det = fmaf(sxx, syy, -(sxy * sxy));
      const float rdet = __builtin_amdgcn_rcpf(det);
      const float rsxx = __builtin_amdgcn_rcpf(sxx);
      s_rc[slot][l] = make_float4(__builtin_amdgcn_sqrtf(-kHalfLog2e * sxx * rdet),
                                  ra * G.flux * pg[5] * kInv2Pi * __builtin_amdgcn_rsqf(det), -sxy * rsxx,
                                  kHalfLog2e * rsxx);
    }
  }

  // Fractional-shift phases (shift theorem): exp(-2 pi i (fx nu + fy om)).
  // Every lane evaluates the y phase of row l and one x phase: lanes h = 0
  // that of column c, lanes h = 1 that of nu = +1/2 (the Nyquist column).
  // The h = 1 lane of a pair takes its column's phase from its neighbour;
  // omega = -1/2 is the conjugate of row W/2 (omega = +1/2).
  float sy, cy;
  sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
  if constexpr (!LZ) {
    // The integer part of the y centre goes into the phase as well:
    // exp(-2 pi i n_y k_y / W) for row k_y = l (mod W) is an exact table
    // entry.  The stamp then leaves the transforms in output row order, and
    // only its columns are rolled at the store.
    const float2 ti = twiddle_rt<-1, W>(G.ny * l);
    const float c2 = fmaf(cy, ti.x, -(sy * ti.y)), s2 = fmaf(cy, ti.y, sy * ti.x);
    cy = c2;
    sy = s2;
  }
  float sxa, cxa;
  sincospi_poly(h ? -G.fx : -2.f * G.fx * nu, &sxa, &cxa);
  const float sx = pair_even(sxa), cx = pair_even(cxa);
  const float sxh = stamp_lane1<W>(sxa), cxh = stamp_lane1<W>(cxa);  // nu = +1/2
  const float fs = G.flux * (1.f / ((float)W * (float)W));
  const float2 pxF = make_float2(fs * cx, fs * sx);
  s_py[slot][l] = make_float2(cy, sy);
  if (l == W / 2) s_py[slot][W] = make_float2(cy, -sy);
  {
    const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
    const bool corner = (l == W / 2);
    const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
    const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
    const float2 plus = cadd(cscale(pyA, SN[0]), cscale(pyB, SN[1]));
    const float2 minus = cadd(cscale(pyA, SN[1]), cscale(pyB, SN[0]));
    const float2 inner = cadd(cmul(eM, plus), cmul(eP, minus));
    s_nyq[slot][l] = cmul(cscale(psfN, 0.5f * fs), inner);
  }
  __syncthreads();

  float2 Z[M];
  static_for<0, M>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    float2 P;
    if constexpr (kPsfStream) P = psfm[m * W + l];
    else P = Pm[m];
    if constexpr (2 * m == W / 2) {
      const float2 q0 = s_py[slot][W / 2 + h];
      const float2 pyA = h ? q0 : cscale(q0, 0.5f);
      const float2 pyB = h ? make_float2(0.f, 0.f) : cscale(s_py[slot][W], 0.5f);
      Z[m] = cmul(cmul(P, pxF), cadd(cscale(pyA, S[m]), cscale(pyB, S[M])));
    } else {
      Z[m] = cscale(cmul(cmul(P, s_py[slot][2 * m + h]), pxF), S[m]);
    }
    if constexpr (kPsfStream && m % 16 == 15) __builtin_amdgcn_sched_barrier(0);  // bounds the loads in flight
  });
  if (c == 0) {  // column 0 carries the Nyquist column as its imaginary part
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 xn = s_nyq[slot][2 * m + h];
      Z[m] = make_float2(Z[m].x - xn.y, Z[m].y + xn.x);
    });
  }
  fft<M, +1>(Z);

  // ---------------------------------------------------------------- row phase
  constexpr int NC = W / 2;
  constexpr int QC = W / 4;  // columns per transpose pass
  const int y = l;
  const int jr = y & (M - 1);
  const float2 tw = twiddle_rt<+1, W>(y);
  float2 X[NC + 1];
  static_for<0, 2>([&](auto pp) {
    constexpr int pass = decltype(pp)::value;
    if (c / QC == pass) {
      static_for<0, M>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        s_t1[slot][j * T1S + (l - 2 * QC * pass)] = Z[j];
      });
    }
    __syncthreads();
    static_for<0, QC>([&](auto cc) {
      constexpr int cl = decltype(cc)::value;
      constexpr int cI = pass * QC + cl;
      const float2 e0 = s_t1[slot][jr * T1S + 2 * cl];
      const float2 e1 = s_t1[slot][jr * T1S + 2 * cl + 1];
      const float2 v = cfma(tw, e1, e0);
      if constexpr (cI == 0) {
        X[0] = make_float2(v.x, 0.f);
        X[NC] = make_float2(v.y, 0.f);
      } else {
        X[cI] = v;
      }
    });
    __syncthreads();
  });
  // complex-to-real: R[k] = (X[k] + conj X[W/2-k]) + i w^k (X[k] - conj X[W/2-k]),
  // w = exp(2 pi i / W).  Bins k and W/2-k share s = X[k] + conj X[W/2-k] and
  // t = w^k (X[k] - conj X[W/2-k]):  R[k] = s + i t,  R[W/2-k] = conj(s) + i conj(t).
  float2 R[NC];
  static_for<0, NC / 2 + 1>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    float2 lo, hi;
    c2r_pair<+1, W, k>(X[k], cconj(X[NC - k]), lo, hi);
    R[k] = lo;
    if constexpr (k != 0 && 2 * k != NC) R[NC - k] = hi;
  });
  fft<NC, +1>(R);

  // ---------------------------------------------------------------- real space + store
  // Output pixel (Y, X = l) is pixel ((Y - ny) mod W, (X - nx) mod W) of the
  // fractional-offset Fourier image: the integer shift is a cyclic roll.  Pass
  // q stages source rows q W/2 .. q W/2 + W/2 - 1 in LDS; they land on output
  // rows (q W/2 + r + ny) mod W.
  float* st = reinterpret_cast<float*>(&s_t1[slot][0]);
  const float dx = (float)l - G.x0 - pg[0];
  const float dyc = -G.y0 - pg[1];
  float* outp = p.out + (live ? stamp : 0) * (int64_t)(W * W);
  if constexpr (LZ) {
    static_assert(W <= 64, "the fused shift keeps a whole column per lane");
    {
      // Lanczos-3 shift by the fractional position, fused into the store: a
      // lane keeps its whole output column (W <= 64), so the stamp makes one
      // trip to memory.  The tile is in output order (the integer shift went
      // into the phase).  The real-space components are added to the rows
      // first (the shift applies to the whole stamp), the rows are filtered
      // along x in the row-owning lane and written to the LDS tile, and the
      // columns are filtered along y in registers as the tile's rows are
      // read.  Taps outside the stamp have weight zero.
      if (rmask != 0) {
        // Real-space components along this lane's row: the exponent is a
        // quadratic in the column x with per-row coefficients, two FMAs per
        // pixel.
        const float dy = (float)y + dyc;
        const float dx0 = -G.x0 - pg[0];  // dx of column 0
        for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
          const float2 rs = s_rs[slot][__builtin_ctz(mk)];
          const float v = rs.x, ra = rs.y;
          const float sxx = fmaf(v, G.b11, pg[2]);
          const float sxy = fmaf(v, G.b12, pg[3]);
          const float syy = fmaf(v, G.b22, pg[4]);
          const float det = fmaf(sxx, syy, -(sxy * sxy));
          const float rdet = __builtin_amdgcn_rcpf(det);
          const float ampr = ra * G.flux * pg[5] * kInv2Pi * __builtin_amdgcn_rsqf(det);
          // Along this lane's row (dy fixed) the quadratic form is
          // dy^2 / syy + (syy / det) (dx - (sxy / syy) dy)^2, completed about
          // the conditional mean so that no large terms cancel near the peak:
          // with dx = x + dx0 the exponent is k - u^2, u = g (x + m).
          const float rsyy = __builtin_amdgcn_rcpf(syy);
          const float g = __builtin_amdgcn_sqrtf(-kHalfLog2e * syy * rdet);
          const float k0 = kHalfLog2e * dy * dy * rsyy;
          const float gm = g * fmaf(-sxy * rsyy, dy, dx0);
          static_for<0, W / 2>([&](auto xx) {
            constexpr int x = 2 * decltype(xx)::value;  // two columns at a time
            const float u0 = fmaf(g, (float)x, gm);
            const float u1 = fmaf(g, (float)(x + 1), gm);
            R[x >> 1].x = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u0, u0, k0)), R[x >> 1].x);
            R[x >> 1].y = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u1, u1, k0)), R[x >> 1].y);
          });
        }
      }
      // x filter of this lane's row, with every lane active (in the staging
      // passes below only half the lanes write, and arithmetic there would
      // be issued once per pass)
      float hrow[W];
      static_for<0, W>([&](auto xx) {
        constexpr int x = decltype(xx)::value;
        float hsum = 0.f;
        static_for<0, 6>([&](auto dd) {
          constexpr int d = decltype(dd)::value;
          constexpr int xs = x + d - 3;
          if constexpr (xs >= 0 && xs < W) hsum = fmaf(wxn[d], (xs & 1) ? R[xs >> 1].y : R[xs >> 1].x, hsum);
        });
        hrow[x] = hsum;
      });
      float acc[W];
      static_for<0, W>([&](auto tt) { acc[decltype(tt)::value] = 0.f; });
      static_for<0, 2>([&](auto qq) {
        constexpr int q = decltype(qq)::value;
        if (y / C::HR == q) {
          int row = (y - q * C::HR) * (W + 1);
          asm volatile("" : "+v"(row));
          static_for<0, W>([&](auto xx) {
            constexpr int x = decltype(xx)::value;
            st[row + x] = hrow[x];
          });
        }
        __syncthreads();
        static_for<0, C::HR>([&](auto rr) {
          constexpr int sr = q * C::HR + decltype(rr)::value;  // source row
          const float v = st[(sr - q * C::HR) * (W + 1) + l];
          static_for<0, 6>([&](auto dd) {
            constexpr int d = decltype(dd)::value;
            constexpr int t = sr - d + 3;  // output row fed through tap d
            if constexpr (t >= 0 && t < W) acc[t] = fmaf(wy[d], v, acc[t]);
          });
          // Output row t is complete once its sources t - 3 .. t + 2 within
          // the stamp are in; the last two rows after the final source row.
          constexpr int done = sr - 2;
          if constexpr (done >= 0) {
            if (live) __builtin_nontemporal_store(acc[done], outp + done * W + l);
          }
          __builtin_amdgcn_sched_barrier(0);
        });
        __syncthreads();
      });
      if (live) {
        __builtin_nontemporal_store(acc[W - 2], outp + (W - 2) * W + l);
        __builtin_nontemporal_store(acc[W - 1], outp + (W - 1) * W + l);
      }
    }
  } else {
    const int colsrc = (l - G.nx) & (W - 1);
    static_for<0, 2>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      if (y / C::HR == q) {
        int row = (y - q * C::HR) * (W + 1);
        asm volatile("" : "+v"(row));  // one base address; the 2n offsets stay immediate
        static_for<0, NC>([&](auto nn) {
          constexpr int n = decltype(nn)::value;
          st[row + 2 * n] = R[n].x;
          st[row + 2 * n + 1] = R[n].y;
        });
      }
      __syncthreads();
      float val[C::HR];
      static_for<0, C::HR>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        val[r] = st[r * (W + 1) + colsrc];
      });
      if (rmask != 0) {
        for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
          const float4 rc = s_rc[slot][__builtin_ctz(mk)];  // LDS, not global: no wait on the stores above
          // Along this lane's column (dx fixed) the quadratic form is
          // dx^2 / sxx + (sxx / det) (dy - (sxy / sxx) dx)^2: the square is
          // completed about the conditional mean, so the exponent stays a
          // difference of small terms near the peak whatever the tile row
          // (an expansion about the tile's first row cancels terms of size
          // (W/2)^2 / syy there).  With dy = dyq + r the exponent is
          // k - u^2, u = g (r + m): two FMAs with an immediate r.
          const float g = rc.x, ampr = rc.y;
          const float k0 = rc.w * dx * dx;
          const float dyq = (float)(q * C::HR) + dyc;
          const float gm = g * fmaf(rc.z, dx, dyq);
          // two rows at a time, so that each exponential has an independent
          // instruction between it and its use
          static_for<0, C::HR / 2>([&](auto rr) {
            constexpr int r = 2 * decltype(rr)::value;
            const float u0 = fmaf(g, (float)r, gm);
            const float u1 = fmaf(g, (float)(r + 1), gm);
            val[r] = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u0, u0, k0)), val[r]);
            val[r + 1] = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u1, u1, k0)), val[r + 1]);
          });
        }
      }
      if (live) {
        if (p.flags & kAccumulate) {
          static_for<0, C::HR>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            float* rowp = outp + (q * C::HR + r) * W;
            __builtin_nontemporal_store(val[r] + rowp[l], &rowp[l]);
          });
        } else {
          static_for<0, C::HR>([&](auto rr) {
            constexpr int r = decltype(rr)::value;
            __builtin_nontemporal_store(val[r], outp + (q * C::HR + r) * W + l);  // streamed output
          });
        }
      }
      __syncthreads();
    });
  }
  if (live && !G.ok && l == 0) atomicAdd(p.invalid, 1ull);
}

template <int W, bool EIG, bool LZ, bool PT>
static hipError_t launch_small(const RenderArgs& args, hipStream_t stream) {
  using C = SmallCfg<W, EIG>;
  constexpr int64_t kMaxBlocks = 1 << 30;
  RenderArgs p = args;
  int64_t done = 0;
  while (done < args.n) {
    const int64_t chunk = std::min<int64_t>(args.n - done, kMaxBlocks * C::SPB);
    p.x = args.x + done;
    p.y = args.y + done;
    p.flux = args.flux + done;
    p.r_e = args.r_e + done;
    p.e1 = args.e1 + done;
    p.e2 = args.e2 + done;
    p.mix_id = args.mix_id ? args.mix_id + done : nullptr;
    p.out = args.out + done * (int64_t)W * W;
    p.psf_px = args.psf_px ? args.psf_px + done : nullptr;
    p.psf_py = args.psf_py ? args.psf_py + done : nullptr;
    p.psf_id = args.psf_id ? args.psf_id + done : nullptr;
    p.n = chunk;
    const unsigned blocks = (unsigned)((chunk + C::SPB - 1) / C::SPB);
    hipLaunchKernelGGL((render_small_kernel<W, EIG, LZ, PT>), dim3(blocks), dim3(C::BLOCK), 0, stream, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

template <int W>
hipError_t launch_render_small(const RenderArgs& args, hipStream_t stream) {
  const bool lz = (W <= 64) && (args.flags & kLanczos3);
  if (args.psf_id) {  // per-galaxy constant PSFs (eig_J == 0)
    if (args.eig_J > 0) return hipErrorInvalidValue;
    if constexpr (W <= 64) {
      if (lz) return launch_small<W, false, true, true>(args, stream);
    }
    return launch_small<W, false, false, true>(args, stream);
  }
  if constexpr (W <= 64) {
    if (lz)
      return args.eig_J > 0 ? launch_small<W, true, true, false>(args, stream)
                            : launch_small<W, false, true, false>(args, stream);
  }
  return args.eig_J > 0 ? launch_small<W, true, false, false>(args, stream)
                        : launch_small<W, false, false, false>(args, stream);
}

template hipError_t launch_render_small<16>(const RenderArgs&, hipStream_t);
template hipError_t launch_render_small<32>(const RenderArgs&, hipStream_t);
template hipError_t launch_render_small<64>(const RenderArgs&, hipStream_t);
template hipError_t launch_render_small<128>(const RenderArgs&, hipStream_t);

}  // namespace gfc
