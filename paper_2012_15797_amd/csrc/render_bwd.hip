// Adjoint of the forward render for W = 16, 32, 64, 128 (Lang 2020, Section
// 2, steps 3-8, differentiated).
//
// For a loss L with upstream gradient g = dL/dI, the Fourier-path part is
// evaluated in the frequency domain:
//   <g, I_F> = W^-2 sum_k X[k] conj(G[k]),   G = DFT(g),
// so with Gamma0[k] = h(k_x) W^-2 P_hat[k] conj(G[k]) (h = 1 on the columns
// k_x = 0, W/2 and 2 elsewhere, summing over the half spectrum) and U0 =
// Gamma0 * (fractional-shift phase), each parameter's derivative is a sum over
// bins of Re(U0 * dS/dtheta), where S = sum_i w_i A_i exp(-2 pi^2 v_i q_B) is
// the real mixture sum.  Every component shares the shape matrix B (C_i =
// v_i B), so the shape derivatives need only S and S1 = sum_i w_i A_i v_i E_i
// per bin.  The integer part of the centre is removed by un-rolling g.  The
// real-space part is accumulated pixel by pixel.  Per-component sums feed the
// amplitude gradients and the routing-weight terms of the smooth ramp.
//
// Each stamp is handled by W lanes, as in the forward kernel:
//  load        lane = output column: real-space sums, g un-rolled into LDS
//  row R2C     lane = row: real-to-complex forward transform (W/2-point FFT)
//  column DFT  lane (c, h): decimation in frequency, rows k_y = 2m + h
//  bins        exponentials per component, accumulations, lane reductions
//  chain rule  B -> (log r_e, e1, e2) and the routing weights, one lane.
#include <map>
#include <mutex>

#include "gfc_device.hpp"
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"
#include "bwd_common.hpp"
#include "gfc_trace.hpp"

namespace gfc {

template <int W>
struct BwdCfg {
  static constexpr int M = W / 2;
  static constexpr int BLOCK = W < 64 ? 64 : W;
  static constexpr int SPB = BLOCK / W;
  static constexpr int TS = W + 2;            // floats per row of the g tile / float2 per row of Gr is W/2+1
  static constexpr int TN = W * (W + 2);      // floats per stamp
  // Floats from one stamp's tile to the next.  At W = 16 two stamps share
  // each 32-lane half of a wavefront, whose 4-byte LDS accesses are served
  // together: a stride of 16 (mod 32) puts the two stamps in different banks.
  static constexpr int TNP = W < 32 ? TN + 16 : TN;
  static constexpr int CH = W <= 64 ? W : 32; // rows per load chunk
  static constexpr int NP = M + 3;            // evaluation points per lane
  // points per block of the component loop: 35 points in blocks of 12, 12, 11 at 64 (blocks
  // of 18 spill), 67 in blocks of 23, 22, 22 at 128 (in the accumulation registers there;
  // one block of 67 spills to memory)
  static constexpr int PB = M <= 16 ? NP : (W == 128 ? 23 : 12);
  static constexpr int WPE = W == 16 ? 3 : (W <= 64 ? 2 : 1);  // occupancy target (waves per SIMD)
};

// Sum over the W lanes of one stamp; every lane of the stamp receives the total.
// Fixed butterfly order (deterministic).  For W = 128 the two wavefronts meet
// in LDS.
template <int W>
__device__ __forceinline__ float seg_sum(float v, float* s_x2) {
  constexpr int LIM = W < 64 ? W : 64;
#pragma unroll
  for (int o = 1; o < LIM; o <<= 1) v += __shfl_xor(v, o);
  if constexpr (W == 128) {
    const int wv = (threadIdx.x >> 6) & 1;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_x2[wv] = v;
    __syncthreads();
    v = s_x2[0] + s_x2[1];
  }
  return v;
}

// Five such sums with one meeting in LDS for W = 128.
template <int W>
__device__ __forceinline__ void seg_sum5(float& a, float& b, float& c, float& d, float& e, float* s_x10) {
  constexpr int LIM = W < 64 ? W : 64;
#pragma unroll
  for (int o = 1; o < LIM; o <<= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c += __shfl_xor(c, o);
    d += __shfl_xor(d, o);
    e += __shfl_xor(e, o);
  }
  if constexpr (W == 128) {
    const int wv = (threadIdx.x >> 6) & 1;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      s_x10[wv] = a;
      s_x10[2 + wv] = b;
      s_x10[4 + wv] = c;
      s_x10[6 + wv] = d;
      s_x10[8 + wv] = e;
    }
    __syncthreads();
    a = s_x10[0] + s_x10[1];
    b = s_x10[2] + s_x10[3];
    c = s_x10[4] + s_x10[5];
    d = s_x10[6] + s_x10[7];
    e = s_x10[8] + s_x10[9];
  }
}

template <int W>
__global__ void __launch_bounds__(BwdCfg<W>::BLOCK) __attribute__((amdgpu_waves_per_eu(BwdCfg<W>::WPE)))
render_bwd_small_kernel(RenderArgs p, const float* __restrict__ gout, float* __restrict__ grad_params,
                        float* __restrict__ amp_part) {
  using C = BwdCfg<W>;
  constexpr int M = C::M;
  constexpr int NP = C::NP;
  constexpr int TS = C::TS;
  __shared__ float s_tile[C::SPB][C::TNP];
  __shared__ float2 s_py[C::SPB][W + 2];
  __shared__ float2 s_nyq[C::SPB][W];
  __shared__ float s_racc[C::SPB][kKmax][6];
  __shared__ float4 s_cmp[C::SPB][kKmax];  // per component: v, w A, w A v (zero when unused)
  __shared__ float s_x2[10];

  // with one stamp per workgroup the stamp index is uniform (scalar)
  const int l = C::SPB == 1 ? (int)threadIdx.x : (int)threadIdx.x % W;
  const int slot = C::SPB == 1 ? 0 : (int)threadIdx.x / W;
  const int64_t stamp = (int64_t)blockIdx.x * C::SPB + slot;
  const bool live = stamp < p.n;
  const int64_t gidx = live ? stamp : p.n - 1;
  Galaxy G = load_galaxy<W>(p, gidx);
  if constexpr (C::SPB == 1) {
    make_uniform(G);
  }
  const float* amp = p.amp + G.table * kKmax;
  const float* var = p.var + G.table * kKmax;
  const float trB = G.b11 + G.b22;
  const int kloop = (C::SPB == 1) ? G.K : p.kmax;

  // per-component constants of the Fourier sums, computed once per stamp:
  // v, w A, w A v and w (w = 0 past the table's K).  A component with A = 0
  // still needs its sums: dL/dA does not depend on A.
  bool real_share = false;  // lane k < K of each wavefront: component k has a real-space share
  {
    const int k = l & 63;
    if (k < kKmax) {
      const float v = var[k];
      const bool in = k < G.K;
      const float w = in ? route_weight<W>(v * trB, p.flags) : 0.f;
      const float wa = w * (in ? amp[k] : 0.f);
      if (l < kKmax) s_cmp[slot][l] = make_float4(v, wa, wa * v, w);
      real_share = in && w < 1.f;
    }
  }

  // routing: components with a real-space share (whatever their amplitude),
  // from the lanes' weights
  unsigned rmask = 0;
  if constexpr (C::SPB == 1) {
    rmask = (unsigned)__ballot(real_share) & ((1u << kKmax) - 1u);
  } else {  // this stamp's W lanes of the ballot
    const unsigned long long rb = __ballot(real_share);
    rmask = (unsigned)(rb >> ((int)__lane_id() & ~(W - 1))) & ((1u << kKmax) - 1u);
  }

  // ------------------------------------------------------------ load + real space
  const float* gp = gout + gidx * (int64_t)(W * W);
  float* tile = s_tile[slot];
  {
    const float dx = (float)l - G.x0 - p.pg[0];
    const int coldst = (l - G.nx) & (W - 1);
    for (int k = 0; k < kKmax; ++k) {
      if (l < 6) s_racc[slot][k][l] = 0.f;
    }
    for (int r0 = 0; r0 < W; r0 += C::CH) {
      float gv[C::CH];
      static_for<0, C::CH>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        gv[r] = gp[(r0 + r) * W + l];
        tile[((r0 + r - G.ny) & (W - 1)) * TS + coldst] = gv[r];
      });
      for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
        const int k = __builtin_ctz(mk);
        const float v = var[k];
        const float sxx = fmaf(v, G.b11, p.pg[2]);
        const float sxy = fmaf(v, G.b12, p.pg[3]);
        const float syy = fmaf(v, G.b22, p.pg[4]);
        const float det = fmaf(sxx, syy, -(sxy * sxy));
        const float rdet = __builtin_amdgcn_rcpf(det);
        const float ixy = -sxy * rdet, iyy = sxx * rdet;
        const float nrm = kInv2Pi * __builtin_amdgcn_rsqf(det);
        const float dy0 = (float)r0 - G.y0 - p.pg[1];
        // Along this lane's column, z = S^-1 (dx, dy) has zy = ixy dx + iyy dy
        // and zx = al + be zy with al = dx / sxx, be = -sxy / sxx, and the
        // quadratic form is q = dx al + zy^2 / iyy.  So the column needs the
        // moments sum g N zy^p (p = 0, 1, 2) only, with the log2 of
        // nrm exp(-q/2) as c0 + c2 zy^2 (the normalisation folded in).
        const float rsxx = __builtin_amdgcn_rcpf(sxx);
        const float al = dx * rsxx, be = -sxy * rsxx;
        const float zy0 = fmaf(iyy, dy0, ixy * dx);
        const float c0 = fmaf(kHalfLog2e * al, dx, __builtin_amdgcn_logf(nrm));
        const float c2 = kHalfLog2e * __builtin_amdgcn_rcpf(iyy);
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
        static_for<0, C::CH>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const float zy = fmaf(iyy, (float)r, zy0);
          const float gn = gv[r] * __builtin_amdgcn_exp2f(fmaf(c2 * zy, zy, c0));
          const float gz = gn * zy;
          m0 += gn;
          m1 += gz;
          m2 = fmaf(gz, zy, m2);
        });
        // sum g N (1, zx, zy, zx^2, zx zy, zy^2) from the moments
        float a0 = m0, ay = m1, ayy = m2;
        float ax = fmaf(be, m1, al * m0);
        float axy = fmaf(be, m2, al * m1);
        float axx = fmaf(be, axy, al * ax);
        a0 = seg_sum<W>(a0, s_x2);
        seg_sum5<W>(ax, ay, axx, axy, ayy, s_x2);
        if (l == 0) {
          s_racc[slot][k][0] += a0;
          s_racc[slot][k][1] += ax;
          s_racc[slot][k][2] += ay;
          s_racc[slot][k][3] += axx;
          s_racc[slot][k][4] += axy;
          s_racc[slot][k][5] += ayy;
        }
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------ row R2C (lane = row y)
  // Gr2[k] = 2 sum_x g[y][x] exp(-2 pi i k x / W), k = 0..W/2.
  {
    const int y = l;
    float2 Zr[M];
    static_for<0, M>([&](auto nn) {
      constexpr int n = decltype(nn)::value;
      Zr[n] = make_float2(tile[y * TS + 2 * n], tile[y * TS + 2 * n + 1]);
    });
    fft<M, -1>(Zr);
    __syncthreads();  // the tile is rewritten as Gr2 rows below
    float2* gr = reinterpret_cast<float2*>(tile);  // [W][W/2 + 1]
    static_for<0, M / 2 + 1>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      constexpr int kc = (M - k) % M;  // Zr[W/2] is Zr[0]
      const float2 a = Zr[k], b = cconj(Zr[kc]);
      const float2 e2 = cadd(a, b);
      const float2 o2 = rot90<-1>(csub(a, b));      // -i (a - b)
      // t2 = exp(-2 pi i k / W) o2 = r u (TwFactor): e2 +- t2 as FMAs
      using TF = TwFactor<-1, W, k>;
      const float2 u = TF::unit(o2);
      if constexpr (k == 0) {
        // Gr2[0] and Gr2[W/2] are real: stored packed as (Gr2[0], Gr2[W/2]) in
        // column 0, which the column DFT transforms as one complex column
        gr[y * (M + 1)] = make_float2(e2.x + u.x, e2.x - u.x);
      } else {
        gr[y * (M + 1) + k] = make_float2(fmaf(TF::r, u.x, e2.x), fmaf(TF::r, u.y, e2.y));
        if constexpr (2 * k != M) gr[y * (M + 1) + (M - k)] = make_float2(fmaf(-TF::r, u.x, e2.x), fmaf(TF::r, u.y, -e2.y));
      }
    });
  }
  __syncthreads();

  // ------------------------------------------------------------ column DFT (lane (c, h))
  const int c = l >> 1, h = l & 1;
  const float2* gr = reinterpret_cast<const float2*>(tile);
  float2 Gk[M];  // 2 G[k_y = 2m + h][c]   (c = 0: packed with column W/2)
  {
    const float sg = h ? -1.f : 1.f;
    static_for<0, M>([&](auto yy) {
      constexpr int yq = decltype(yy)::value;
      const float2 a = gr[yq * (M + 1) + c];  // c = 0: the packed (k_x = 0, k_x = W/2) pair
      const float2 b = gr[(yq + M) * (M + 1) + c];
      const float2 v = make_float2(fmaf(sg, b.x, a.x), fmaf(sg, b.y, a.y));
      const float2 tw = twiddle<-1, W, yq>(v);  // exp(-2 pi i yq / W) v
      Gk[yq] = h ? tw : v;
    });
    fft<M, -1>(Gk);
  }
  // Unpack the packed column: Z = G0 + i GN, with G0 and GN Hermitian in k_y.
  if (c == 0) {
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      s_nyq[slot][2 * m + h] = Gk[m];
    });
  }
  __syncthreads();
  float2 GN;  // 2 G[k_y = l][W/2]
  {
    const float2 za = s_nyq[slot][l], zb = cconj(s_nyq[slot][(W - l) & (W - 1)]);
    const float2 d = csub(za, zb);
    GN = make_float2(0.5f * d.y, -0.5f * d.x);  // (za - conj zb) / (2 i)
  }
  if (c == 0) {
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 zb = cconj(s_nyq[slot][(W - 2 * m - h) & (W - 1)]);
      Gk[m] = cscale(cadd(Gk[m], zb), 0.5f);
    });
  }

  // ------------------------------------------------------------ phases and U0 per point
  const float nu = (float)c * (1.f / W);
  const float hW = (float)h * (1.f / W);
  // Each lane evaluates the y phase of row l and one x phase (lanes h = 0:
  // column c; lanes h = 1: nu = +1/2), as in the forward kernel.
  const float omN = (l < W / 2) ? (float)l * (1.f / W) : (l == W / 2 ? 0.5f : (float)(l - W) * (1.f / W));
  float sy, cy, sxa, cxa;
  sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
  sincospi_poly(h ? -G.fx : -2.f * G.fx * nu, &sxa, &cxa);
  const float sx = pair_even(sxa), cx = pair_even(cxa);
  const float sxh = stamp_lane1<W>(sxa), cxh = stamp_lane1<W>(cxa);
  s_py[slot][l] = make_float2(cy, sy);
  if (l == W / 2) s_py[slot][W] = make_float2(cy, -sy);  // omega = -1/2: conjugate of omega = +1/2
  __syncthreads();

  // Points: m = 0..M-1 (column c, row 2m+h), M (omega = -1/2 twin of the
  // Nyquist row), M+1, M+2 (Nyquist column row l: nu = +-1/2).  U0 already
  // carries the Nyquist means.  The corner's omega = -1/2 twins fold into
  // M+1 and M+2 (see below).
  float ure[NP], uim[NP];
  // (nu, omega) of point j
  auto point = [&](auto jj, float& n_, float& o_) {
    constexpr int j = decltype(jj)::value;
    if constexpr (j < M) {
      n_ = nu;
      if constexpr (2 * j < W / 2) o_ = (float)(2 * j) * (1.f / W) + hW;
      else if constexpr (2 * j == W / 2) o_ = h ? (float)(W / 2 + 1 - W) * (1.f / W) : 0.5f;
      else o_ = (float)(2 * j - W) * (1.f / W) + hW;
    } else if constexpr (j == M) {
      n_ = nu;
      o_ = -0.5f;
    } else {
      n_ = (j - M) & 1 ? 0.5f : -0.5f;
      o_ = omN;
    }
  };
  {
    // h(k_x) / W^2 with h = 1 on column 0 and 2 elsewhere, halved for the factor 2 in Gk
    const float colw = (c == 0 ? 0.5f : 1.f) / ((float)W * (float)W);
    const float2 px = make_float2(cx * colw, sx * colw);  // the column's phase, with its weight
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 P = p.psf_main[m * W + l];
      const float2 gp2 = cmul(cmulc(P, Gk[m]), px);   // P conj(G) x phase x weight
      float2 u;
      if constexpr (2 * m == W / 2) {
        const float2 q0 = s_py[slot][W / 2 + h];
        const float2 pyA = h ? q0 : cscale(q0, 0.5f);
        u = cmul(gp2, pyA);
        const float2 pyB = h ? make_float2(0.f, 0.f) : cscale(s_py[slot][W], 0.5f);
        const float2 ux = cmul(gp2, pyB);
        ure[M] = ux.x;
        uim[M] = ux.y;
      } else {
        u = cmul(gp2, s_py[slot][2 * m + h]);
      }
      ure[m] = u.x;
      uim[m] = u.y;
      if constexpr (m % 8 == 7) __builtin_amdgcn_sched_barrier(0);  // bounds the PSF loads in flight
    });
    // Nyquist column, row l: h = 1, halved for the factor 2 in GN, and the
    // weight 1/2 of each of the nu = +-1/2 representatives
    const float2 gamN = cscale(cmulc(p.psf_nyq[l], GN), 0.25f / ((float)W * (float)W));
    const bool corner = (l == W / 2);
    const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
    const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
    const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
    const float2 u1 = cmul(cmul(gamN, eM), pyA), u2 = cmul(cmul(gamN, eP), pyA);
    const float2 u3 = cmul(cmul(gamN, eM), pyB), u4 = cmul(cmul(gamN, eP), pyB);
    // The mixture transform is even, so at the corner (omN = +1/2) the twin
    // (-1/2, -1/2) has the transform of (+1/2, +1/2) and (+1/2, -1/2) that of
    // (-1/2, +1/2).  A twin's terms are those of its partner with (nu, omega)
    // negated: its real part adds to the partner's, its imaginary part (which
    // multiplies nu or omega) subtracts.  Elsewhere u3 = u4 = 0.
    ure[M + 1] = u1.x + u4.x; uim[M + 1] = u1.y - u4.y;  // (+1/2, omN)
    ure[M + 2] = u2.x + u3.x; uim[M + 2] = u2.y - u3.y;  // (-1/2, omN)
  }

  // ------------------------------------------------------------ component loop
  float ax = 0.f, ay = 0.f, a11 = 0.f, a12 = 0.f, a22 = 0.f;
  // per-lane p_k partials [kKmax][PKS] in the g tile, which the column DFT
  // has finished reading.  The row stride W + LPK makes the reduction below
  // free of bank conflicts.
  constexpr int LPK = W / kKmax;  // lanes per component in that reduction
  static_assert(LPK >= 1 && W % kKmax == 0, "components share the stamp's lanes evenly");
  constexpr int PKS = W + LPK;
  float* s_pk = &s_tile[slot][0];
  static_assert(kKmax * PKS <= C::TN, "p_k partials fit in the tile");
  for (int k = 0; k < kKmax; ++k) s_pk[k * PKS + l] = 0.f;
  float m_si = 0.f, m_csi = 0.f, m_r = 0.f, m_cr = 0.f, m_ccr = 0.f;
  // The exponent's quadratic form along this lane's column, expanded about
  // omega = h/W: at omega = c + h/W with a compile-time c it is
  // e0 + c (e1 + c g2), two FMAs with immediates.
  const float g2 = kQ * G.b22, g1 = 2.f * kQ * G.b12 * nu;
  const float e0 = fmaf(hW, fmaf(g2, hW, g1), kQ * G.b11 * nu * nu);
  const float e1 = fmaf(2.f * g2, hW, g1);
  static_for<0, (NP + C::PB - 1) / C::PB>([&](auto bb) {
    constexpr int b0 = decltype(bb)::value * C::PB;
    constexpr int nb = (NP - b0) < C::PB ? (NP - b0) : C::PB;
    float gq[nb], S[nb], S1[nb];
    static_for<0, nb>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      constexpr int jp = b0 + j;
      if constexpr (jp < M && 2 * jp != W / 2) {
        constexpr float cm = (2 * jp < W / 2) ? (float)(2 * jp) * (1.f / W) : (float)(2 * jp - W) * (1.f / W);
        gq[j] = fmaf(cm, fmaf(cm, g2, e1), e0);
      } else {
        float n_, o_;
        point(std::integral_constant<int, jp>{}, n_, o_);
        gq[j] = kQ * fmaf(G.b11 * n_, n_, fmaf(2.f * G.b12 * n_, o_, G.b22 * o_ * o_));
      }
    });
    // Component 0 initialises the sums (every table has one).  With w = 0 it
    // adds zeros to S and S1, and its p_k partial, finite since e <= 1, is
    // only ever multiplied by w or by the ramp slope, both zero then.
    {
      const float4 cp = s_cmp[slot][0];
      float pk = 0.f;
      static_for<0, nb>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const float e = __builtin_amdgcn_exp2f(cp.x * gq[j]);
        S[j] = cp.y * e;
        S1[j] = cp.z * e;
        pk = fmaf(ure[b0 + j], e, pk);
      });
      s_pk[l] += pk;
    }
    // The next component's constants and partial are read one iteration
    // ahead, so that the LDS latency falls behind this component's work.
    float4 cpn = s_cmp[slot][1];
    float pkn = s_pk[PKS + l];
#pragma unroll 2
    for (int k = 1; k < kloop; ++k) {
      // p_k is needed when w_k > 0 (amplitude and ramp terms); w_k = 0 means n_k <= 3,
      // where the ramp slope vanishes too
      const float4 cp = cpn;
      const float pk_before = pkn;
      {  // unconditional, clamped into the arrays (the last read is not used)
        const int kn = min(k + 1, kKmax - 1);
        cpn = s_cmp[slot][kn];
        pkn = s_pk[kn * PKS + l];
      }
      const float v = cp.x, wa = cp.y, wav = cp.z;
      if (cp.w == 0.f) continue;
      float pk = 0.f;
      static_for<0, nb>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const float e = __builtin_amdgcn_exp2f(v * gq[j]);
        S[j] = fmaf(wa, e, S[j]);
        S1[j] = fmaf(wav, e, S1[j]);
        pk = fmaf(ure[b0 + j], e, pk);
      });
      s_pk[k * PKS + l] = pk_before + pk;
    }
    static_for<0, nb>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      constexpr int jp = b0 + j;
      const float si = S[j] * uim[jp];
      const float r1 = S1[j] * ure[jp];
      if constexpr (jp < M && 2 * jp != W / 2) {
        // omega = c + h/W, nu the lane's: the moments of si and r1 in c
        constexpr float cm = (2 * jp < W / 2) ? (float)(2 * jp) * (1.f / W) : (float)(2 * jp - W) * (1.f / W);
        m_si += si;
        m_csi = fmaf(cm, si, m_csi);
        m_r += r1;
        m_cr = fmaf(cm, r1, m_cr);
        m_ccr = fmaf(cm * cm, r1, m_ccr);
      } else {
        float n_, o_;
        point(std::integral_constant<int, jp>{}, n_, o_);
        ax = fmaf(n_, si, ax);
        ay = fmaf(o_, si, ay);
        a11 = fmaf(n_ * n_, r1, a11);
        a12 = fmaf(n_ * o_, r1, a12);
        a22 = fmaf(o_ * o_, r1, a22);
      }
    });
    // Materialise the block's contribution here, so the compiler does not sink
    // the accumulation (and keep this block's sums alive) past later blocks.
    asm volatile("" : "+v"(ax), "+v"(ay), "+v"(a11), "+v"(a12), "+v"(a22));
    asm volatile("" : "+v"(m_si), "+v"(m_csi), "+v"(m_r), "+v"(m_cr), "+v"(m_ccr));
  });
  // the regular points' terms from their moments: with omega = c + h/W,
  // sum nu si, sum omega si, sum nu^2 r1, sum nu omega r1, sum omega^2 r1
  ax = fmaf(nu, m_si, ax);
  ay += fmaf(hW, m_si, m_csi);
  a11 = fmaf(nu * nu, m_r, a11);
  a12 = fmaf(nu, fmaf(hW, m_r, m_cr), a12);
  a22 += fmaf(hW, fmaf(hW, m_r, 2.f * m_cr), m_ccr);
  seg_sum5<W>(ax, ay, a11, a12, a22, s_x2);
  __syncthreads();
  // p_k = sum over the stamp's W partials, fixed order: LPK lanes per
  // component, lane i taking the entries i, i + LPK, ..., then a butterfly
  // over the LPK lanes.
  {
    const int k = l / LPK, i = l % LPK;
    float acc = 0.f;
#pragma unroll
    for (int e = 0; e < W / LPK; ++e) acc += s_pk[k * PKS + i + e * LPK];
#pragma unroll
    for (int o = 1; o < LPK; o <<= 1) acc += __shfl_xor(acc, o);
    if (i == 0) s_pk[k * PKS] = acc;
  }
  __syncthreads();

  // ------------------------------------------------------------ chain rule
  // lane k of the stamp takes component k; the terms are summed over 16 lanes
  // and lane 0 finishes B -> (log r_e, e1, e2)
  {
    // The galaxy is reloaded here, through renewed argument and stamp
    // values, so that neither it nor its addresses hold registers through
    // the loops above.
    const RenderArgs& pc = kernel_args_renewed<RenderArgs>();
    int64_t gi = gidx;
    if constexpr (C::SPB == 1) asm volatile("" : "+s"(gi));
    Galaxy Gc = load_galaxy<W>(pc, gi);
    if constexpr (C::SPB == 1) make_uniform(Gc);
    CompTerms t = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live && l < kKmax)
      t = bwd_component_terms<W>(pc, Gc, l, rmask, s_pk, PKS, &s_racc[slot][0][0], amp_part + gi * kKmax);
    t = sum16(t);
    if (l == 0 && live) bwd_chain_finish<W>(pc, Gc, gi, ax, ay, a11, a12, a22, t, grad_params);
  }
}

// grad_amp[t][k] += sum over galaxies i with table t of amp_part[i][k]
// (amp_part is [n][kKmax] row-major).  Every order below is fixed, so the
// sums are the same from run to run.
//
// Two passes: the galaxies in chunks of kAgChunk, each (chunk, table) block
// summing its rows with kAgRows threads per component (index order within a
// thread, coalesced reads of whole rows) and a fixed tree over the threads;
// then per table the chunk partials the same way.
constexpr int kAgChunk = 128;
constexpr int kAgRows = 256 / kKmax;

__global__ void __launch_bounds__(256) amp_grad_partial(const float* __restrict__ amp_part,
                                                        const int32_t* __restrict__ mix_id, int64_t n, int t0,
                                                        int64_t nchunks, float* __restrict__ partial) {
  const int64_t c = blockIdx.x;
  const int t = t0 + (int)blockIdx.y;
  const int r = threadIdx.x / kKmax, k = threadIdx.x % kKmax;
  const int64_t i1 = min(n, (c + 1) * kAgChunk);
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < kAgChunk / kAgRows; ++j) {  // the loads issue together; the adds stay in index order
    const int64_t i = c * kAgChunk + r + j * kAgRows;
    if (i < i1) {
      const int ti = mix_id ? mix_id[i] : 0;
      if (ti == t) acc += amp_part[i * kKmax + k];
    }
  }
  __shared__ float s[256];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o >= kKmax; o >>= 1) {  // rows r and r + o / kKmax, same component
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < kKmax) partial[((int64_t)t * nchunks + c) * kKmax + threadIdx.x] = s[threadIdx.x];
}

__global__ void __launch_bounds__(256) amp_grad_finish(const float* __restrict__ partial, int64_t nchunks,
                                                       float* __restrict__ grad_amp) {
  const int t = blockIdx.x;
  const int r = threadIdx.x / kKmax, k = threadIdx.x % kKmax;
  float acc = 0.f;
#pragma unroll 8
  for (int64_t c = r; c < nchunks; c += kAgRows) acc += partial[((int64_t)t * nchunks + c) * kKmax + k];
  __shared__ float s[256];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o >= kKmax; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < kKmax) grad_amp[t * kKmax + threadIdx.x] += s[threadIdx.x];
}

// One pass per (table, component), for table counts whose chunk partials
// would take more than 64 MiB: index order within fixed 256-wide strides,
// then a fixed tree.
__global__ void amp_grad_reduce(const float* __restrict__ amp_part, const int32_t* __restrict__ mix_id,
                                int64_t n, float* __restrict__ grad_amp) {
  const int t = blockIdx.x / kKmax, k = blockIdx.x % kKmax;
  __shared__ float s[256];
  float acc = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const int ti = mix_id ? mix_id[i] : 0;
    if (ti == t) acc += amp_part[i * kKmax + k];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad_amp[t * kKmax + k] += s[0];
}

template <int W>
static hipError_t launch_bwd_small(const RenderArgs& args, const float* gout, float* grad_params,
                                   float* amp_part, hipStream_t stream) {
  using C = BwdCfg<W>;
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
    p.n = chunk;
    const unsigned blocks = (unsigned)((chunk + C::SPB - 1) / C::SPB);
    hipLaunchKernelGGL(render_bwd_small_kernel<W>, dim3(blocks), dim3(C::BLOCK), 0, stream, p,
                       gout + done * (int64_t)W * W, grad_params + done * 6, amp_part + done * kKmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace gfc

using namespace gfc;

// Tables whose chunk partials the workspace holds (beyond that they take a
// stream-ordered allocation).
constexpr int kAgWsTables = 16;

static int64_t amp_grad_chunks(int64_t n) { return (n + kAgChunk - 1) / kAgChunk; }

// ws_partial: the workspace's room for kAgWsTables tables' partials.  With
// more tables the partials take a stream-ordered allocation, unless
// may_allocate is false: then the one-pass reduction runs instead.
static hipError_t launch_amp_grad(const float* amp_part, const int32_t* mix_id, int64_t n, int n_tables,
                                  float* grad_amp, float* ws_partial, hipStream_t s, bool may_allocate = true) {
  const int64_t nchunks = amp_grad_chunks(n);
  if ((int64_t)n_tables * nchunks > (int64_t)1 << 20 || (n_tables > kAgWsTables && !may_allocate)) {
    hipLaunchKernelGGL(amp_grad_reduce, dim3(n_tables * kKmax), dim3(256), 0, s, amp_part, mix_id, n, grad_amp);
    return hipGetLastError();
  }
  float* partial = ws_partial;
  hipError_t e = hipSuccess;
  const bool own = n_tables > kAgWsTables;
  if (own) {
    e = hipMallocAsync((void**)&partial, (size_t)n_tables * nchunks * kKmax * sizeof(float), s);
    if (e != hipSuccess) return e;
  }
  constexpr int kMaxY = 65535;  // tables per launch (grid y)
  for (int t0 = 0; t0 < n_tables && e == hipSuccess; t0 += kMaxY) {
    const int nt = std::min(n_tables - t0, kMaxY);
    hipLaunchKernelGGL(amp_grad_partial, dim3((unsigned)nchunks, (unsigned)nt), dim3(256), 0, s, amp_part, mix_id,
                       n, t0, nchunks, partial);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(amp_grad_finish, dim3((unsigned)n_tables), dim3(256), 0, s, partial, nchunks, grad_amp);
    e = hipGetLastError();
  }
  if (own) {
    const hipError_t e2 = hipFreeAsync(partial, s);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

// ---------------------------------------------------------------- allocation-free adjoint
// Scratch of gfc_render_stamps_backward_noalloc, laid out as the workspace of
// gfc_render_stamps_backward for n galaxies: amplitude partials [n][kKmax],
// parameter gradients [n][6] (used when grad_params is NULL), then the
// two-pass reduction's partials for kAgWsTables tables.  Sized for
// GFC_NOALLOC_MAX_GALAXIES; each device holds its own copy (24 MiB) from
// the first context created on it until the process ends.  Every call on a
// device shares that copy, and each call overwrites what it reads, so
// nothing needs clearing between calls.
constexpr int64_t kNoAllocMax = GFC_NOALLOC_MAX_GALAXIES;
constexpr size_t kNoAllocFloats =
    (size_t)kNoAllocMax * (kKmax + 6) + (size_t)kAgWsTables * ((kNoAllocMax + kAgChunk - 1) / kAgChunk) * kKmax;
static __device__ __align__(256) float scratch[kNoAllocFloats];

namespace {
std::mutex g_scratch_mu;
std::map<int, float*> g_scratch_ptr;  // HIP device -> address of that device's `scratch`
}  // namespace

namespace gfc {
// Takes the device address of `scratch` on `device`, which must be current.
// Host code uses only this address: the array's name is a host-side stand-in.
gfc_status noalloc_scratch_setup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return GFC_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the adjoint's scratch array");
  if (!ptr) return fail(GFC_EDEVICE, "the adjoint's scratch array has no device address");
  g_scratch_ptr[device] = static_cast<float*>(ptr);
  return GFC_OK;
}
}  // namespace gfc

static float* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

extern "C" {

size_t gfc_backward_workspace_bytes(int64_t n) {
  return n > 0 ? ((size_t)n * kKmax + 6 * (size_t)n + (size_t)kAgWsTables * amp_grad_chunks(n) * kKmax) * sizeof(float)
               : 0;
}

gfc_status gfc_render_stamps_backward(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix, const gfc_galaxies* gal,
                                      int64_t n, int W, unsigned flags, const float* grad_out,
                                      float* grad_params, float* grad_amp, void* workspace,
                                      void* hip_stream) {
  TraceScope trace("gfc render backward");
  if (psf && psf->J > 0) return fail(GFC_EUNSUPPORTED, "the adjoint takes a constant PSF");
  if (flags & GFC_SHIFT_LANCZOS3) return fail(GFC_EUNSUPPORTED, "the adjoint uses the Fourier-phase shift");
  if (flags & GFC_ACCUMULATE) return fail(GFC_EINVAL, "GFC_ACCUMULATE applies to forward renders");
  RenderArgs a;
  gfc_status st = fill_render_args(ctx, psf, mix, gal, n, W, flags, &a);
  if (st != GFC_OK) return st;
  if (n == 0) return GFC_OK;
  if (!grad_out) return fail(GFC_EINVAL, "null upstream gradient");
  DeviceGuard guard(ctx->device);
  hipStream_t s = (hipStream_t)hip_stream;
  const PsfSpectrum* spec = nullptr;
  st = psf_cache(psf, W, s, &spec);
  if (st != GFC_OK) return st;
  attach_spectrum(&a, spec);
  float* ws = static_cast<float*>(workspace);
  bool own = false;
  hipError_t e = hipSuccess;
  if (!ws) {
    e = hipMallocAsync((void**)&ws, gfc_backward_workspace_bytes(n), s);
    if (e != hipSuccess) return fail(GFC_ENOMEM, "backward workspace allocation failed");
    own = true;
  }
  float* amp_part = ws;
  float* gp = grad_params ? grad_params : ws + (size_t)n * kKmax;
  switch (W) {
    case 16: e = launch_bwd_small<16>(a, grad_out, gp, amp_part, s); break;
    case 32: e = launch_bwd_small<32>(a, grad_out, gp, amp_part, s); break;
    case 64: e = launch_bwd_small<64>(a, grad_out, gp, amp_part, s); break;
    case 128: e = launch_bwd_small<128>(a, grad_out, gp, amp_part, s); break;
    case 256: e = launch_bwd_w256(a, grad_out, gp, amp_part, s); break;
  }
  if (e == hipSuccess && grad_amp)
    e = launch_amp_grad(amp_part, gal->mix_id, n, mix->n_tables, grad_amp, ws + (size_t)n * (kKmax + 6), s);
  if (own) {
    hipError_t e2 = hipFreeAsync(ws, s);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return GFC_OK;
}

gfc_status gfc_render_stamps_backward_noalloc(gfc_ctx* ctx, gfc_psf* psf, const gfc_mix* mix,
                                              const gfc_galaxies* gal, int64_t n, int W, unsigned flags,
                                              const float* grad_out, float* grad_params, float* grad_amp,
                                              void* hip_stream) {
  if (psf && psf->J > 0) return fail(GFC_EUNSUPPORTED, "the adjoint takes a constant PSF");
  if (flags & GFC_SHIFT_LANCZOS3) return fail(GFC_EUNSUPPORTED, "the adjoint uses the Fourier-phase shift");
  if (flags & GFC_ACCUMULATE) return fail(GFC_EINVAL, "GFC_ACCUMULATE applies to forward renders");
  RenderArgs a;
  gfc_status st = fill_render_args(ctx, psf, mix, gal, n, W, flags, &a);
  if (st != GFC_OK) return st;
  if (W > 128) return fail(GFC_EINVAL, "the allocation-free adjoint takes stamp sizes up to 128");
  if (n > kNoAllocMax)
    return fail(GFC_EINVAL, "the allocation-free adjoint takes at most GFC_NOALLOC_MAX_GALAXIES galaxies per call");
  if (n == 0) return GFC_OK;
  if (!grad_out) return fail(GFC_EINVAL, "null upstream gradient");
  DeviceGuard guard(ctx->device);
  const PsfSpectrum* spec = psf_cache_find(psf, W);
  if (!spec) return fail(GFC_EINVAL, "no cached PSF spectrum for this stamp size: call gfc_psf_prepare first");
  attach_spectrum(&a, spec);
  float* ws = noalloc_scratch(ctx->device);
  if (!ws) return fail(GFC_EDEVICE, "the adjoint's scratch array is not set up on this device");
  hipStream_t s = (hipStream_t)hip_stream;
  float* amp_part = ws;
  float* gp = grad_params ? grad_params : ws + (size_t)n * kKmax;
  hipError_t e = hipSuccess;
  switch (W) {
    case 16: e = launch_bwd_small<16>(a, grad_out, gp, amp_part, s); break;
    case 32: e = launch_bwd_small<32>(a, grad_out, gp, amp_part, s); break;
    case 64: e = launch_bwd_small<64>(a, grad_out, gp, amp_part, s); break;
    case 128: e = launch_bwd_small<128>(a, grad_out, gp, amp_part, s); break;
  }
  if (e == hipSuccess && grad_amp)
    e = launch_amp_grad(amp_part, gal->mix_id, n, mix->n_tables, grad_amp, ws + (size_t)n * (kKmax + 6), s,
                        /*may_allocate=*/false);
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return GFC_OK;
}

}  // extern "C"
