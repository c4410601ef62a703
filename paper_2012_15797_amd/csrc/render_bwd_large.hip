// Adjoint of the forward render for 256 x 256 stamps (Lang 2020, Section 2,
// steps 3-8, differentiated); same sums as the W <= 128 adjoint.
//
// One 512-thread workgroup per stamp, with a 264 KB device slab per stamp
// (the half spectrum does not fit in LDS):
//  load       64 rows at a time: the upstream gradient g is un-rolled by the
//             integer centre through LDS and written to the slab as column
//             pairs (g[y][2n], g[y][2n+1]), y fastest; real-space sums are
//             accumulated on the way.
//  row R2C    wavefront pairs own 64 rows; the two wavefronts of a pair take
//             the even and odd outputs of the 128-point complex FFT that the
//             real-to-complex row transform reduces to.
//  column     lane (c, h) with h uniform per wavefront pair: the first
//             radix-4 stage of the 256-point column DFT by decimation in
//             frequency, then a 64-point FFT in registers -> rows 4m + h.
//  bins       per-component exponentials and accumulations as in the
//             smaller adjoint, then fixed-order block reductions and the
//             chain rule on one lane.
#include "bwd_common.hpp"
#include "gfc_device.hpp"
#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

namespace gfc {

namespace bigb {
constexpr int W = 256;
constexpr int D = 4;
constexpr int M = W / D;            // 64 rows per lane in the column phase
constexpr int NC = W / 2;           // 128 regular columns
constexpr int BLOCK = 512;
constexpr int NWAVE = BLOCK / 64;
constexpr int RCH = 64;             // rows per load chunk
constexpr int TS = W + 1;           // floats per LDS tile row
constexpr int SLAB = NC * W;        // float2 per stamp: [y][k_x], column 0 packed with k_x = 128
constexpr int NP = M + 3;
constexpr int PB = 8;
}  // namespace bigb

// Sum over the 512 threads; every thread receives the total (fixed order).
__device__ __forceinline__ float block_sum512(float v, float* s_red /*[8]*/) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < bigb::NWAVE; ++w) t += s_red[w];
  return t;
}

__global__ void __launch_bounds__(bigb::BLOCK)
render_bwd_w256_kernel(RenderArgs p, const float* __restrict__ gout, float* __restrict__ grad_params,
                       float* __restrict__ amp_part, float2* __restrict__ scratch) {
  using namespace bigb;
  __shared__ float s_tile[RCH * TS];
  __shared__ float2 s_py[W + 2];
  __shared__ float2 s_nyq[W];
  __shared__ float s_red[NWAVE];
  __shared__ float s_racc[kKmax][6];
  __shared__ float s_pkw[kKmax][NWAVE];
  __shared__ float4 s_cmp[kKmax];  // per component: v, w A, w A v, w (zero past the table's K)

  const int l = threadIdx.x;
  const int64_t gidx = blockIdx.x;  // the launcher sizes each grid to its chunk
  Galaxy G = load_galaxy<W>(p, gidx);
  make_uniform(G);
  const float* amp = p.amp + G.table * kKmax;
  const float* var = p.var + G.table * kKmax;
  const float trB = G.b11 + G.b22;
  float2* slab = scratch + (int64_t)blockIdx.x * SLAB;
  float2* gT = slab;  // un-rolled g as [n][y] pairs (g[y][2n], g[y][2n+1])

  // Lane k of every wavefront works out component k's route weight once per
  // stamp; the real-space mask is the ballot of w < 1 (whatever A_k: dL/dA_k
  // needs it), and the first wavefront leaves the Fourier-loop constants in LDS.
  unsigned rmask;
  {
    const int k = l & 63;
    float vk = 0.f, wk = 0.f, ak = 0.f;
    bool rs = false;
    if (k < G.K) {
      vk = var[k];
      wk = route_weight<W>(vk * trB, p.flags);
      ak = amp[k];
      rs = wk < 1.f;
    }
    rmask = (unsigned)__ballot(rs) & ((1u << kKmax) - 1u);
    if (l < kKmax) {
      const float wa = wk * ak;
      s_cmp[l] = make_float4(vk, wa, wa * vk, wk);
    }
  }
  if (l < kKmax * 6) (&s_racc[0][0])[l] = 0.f;

  // ------------------------------------------------------------ load + real space
  {
    const int X = l & (W - 1), rh = l >> 8;
    const float dx = (float)X - G.x0 - p.pg[0];
    const float dyc = -G.y0 - p.pg[1];
    const int coldst = (X - G.nx) & (W - 1);
    const float* gp = gout + gidx * (int64_t)(W * W);
    for (int t = 0; t < W / RCH; ++t) {
      const int ybase = (t * RCH + rh * (RCH / 2) + G.ny) & (W - 1);  // output row of local row 0
      const int rwrap = W - ybase;
      float gv[RCH / 2];
      static_for<0, RCH / 2>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        gv[r] = gp[((ybase + r) & (W - 1)) * W + X];
        s_tile[(rh * (RCH / 2) + r) * TS + coldst] = gv[r];
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
        const float dyb = (float)ybase + dyc, dybw = dyb - (float)W;
        // Along this thread's column zy = ixy dx + iyy dy, zx = al + be zy
        // (al = dx / sxx, be = -sxy / sxx) and q = dx al + zy^2 / iyy, so the
        // column needs sum g N zy^p (p = 0, 1, 2) only; log2 of nrm exp(-q/2)
        // is c0 + c2 zy^2.
        const float rsxx = __builtin_amdgcn_rcpf(sxx);
        const float al = dx * rsxx, be = -sxy * rsxx;
        const float zyb = fmaf(iyy, dyb, ixy * dx), zybw = fmaf(iyy, dybw, ixy * dx);
        const float c0 = fmaf(kHalfLog2e * al, dx, __builtin_amdgcn_logf(nrm));
        const float c2 = kHalfLog2e * __builtin_amdgcn_rcpf(iyy);
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
        static_for<0, RCH / 2>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const float zy = fmaf(iyy, (float)r, (r >= rwrap) ? zybw : zyb);
          const float gn = gv[r] * __builtin_amdgcn_exp2f(fmaf(c2 * zy, zy, c0));
          const float gz = gn * zy;
          m0 += gn;
          m1 += gz;
          m2 = fmaf(gz, zy, m2);
        });
        // sum g N (1, zx, zy, zx^2, zx zy, zy^2) from the moments
        float acc[6];
        acc[0] = m0;
        acc[2] = m1;
        acc[5] = m2;
        acc[1] = fmaf(be, m1, al * m0);
        acc[4] = fmaf(be, m2, al * m1);
        acc[3] = fmaf(be, acc[4], al * acc[1]);
        for (int i = 0; i < 6; ++i) {
          const float tot = block_sum512(acc[i], s_red);
          if (l == 0) s_racc[k][i] += tot;
        }
      }
      __syncthreads();
      // tile row r holds un-rolled row t*RCH + r
      {
        const int srl = l & (RCH - 1), xg = l >> 6;
        static_for<0, NC / NWAVE>([&](auto xx) {
          constexpr int xi = decltype(xx)::value;
          const int n = xg * (NC / NWAVE) + xi;
          gT[n * W + t * RCH + srl] = make_float2(s_tile[srl * TS + 2 * n], s_tile[srl * TS + 2 * n + 1]);
        });
      }
      __syncthreads();
    }
  }

  // ------------------------------------------------------------ row R2C
  // Gr2[k] = 2 sum_x g[y][x] exp(-2 pi i k x / W) for k = 0..128, written as
  // X[y][k] into the slab (X[y][0] = Gr2[0] + i Gr2[128], both real).
  const int wv = __builtin_amdgcn_readfirstlane(l >> 6);  // wavefront index (uniform)
  const bool odd = (wv & 1) != 0;
  const int q = odd ? 1 : 0;
  const int y = ((wv >> 1) << 6) | (l & 63);
  // r1[i] = Gr2[k], r2[i] = Gr2[128 - k] for k = 2i + q (i = 0..31); mid = Gr2[64] (q = 0)
  float2 r1[M / 2], r2[M / 2], mid = make_float2(0.f, 0.f);
  auto r2c = [&](auto qq) {
    constexpr int Q = decltype(qq)::value;
    // 128-point DFT Z of z[n] = g[y][2n] + i g[y][2n+1], split by output parity:
    // Z[2k' + Q] = sum_{n<64} a[n] exp(-2 pi i n k' / 64) with
    // a[n] = z[n] + z[n+64] (Q = 0) or (z[n] - z[n+64]) exp(-2 pi i n / 128) (Q = 1)
    float2 a[M];
    static_for<0, M>([&](auto nn) {
      constexpr int n = decltype(nn)::value;
      const float2 z0 = gT[n * W + y], z1 = gT[(n + M) * W + y];
      if constexpr (Q == 0) a[n] = cadd(z0, z1);
      else a[n] = twiddle<-1, 128, n>(csub(z0, z1));
      if constexpr (n % 16 == 15) __builtin_amdgcn_sched_barrier(0);  // bounds the loads in flight
    });
    fft<M, -1>(a);  // a[k'] = Z[2k' + Q]
    // Real-input split, with Z[128 - k] = a[(64 - i) % 64] (Q = 0) or a[63 - i] (Q = 1):
    //   Gr2[k] = e + t, Gr2[128 - k] = conj(e - t),
    //   e = Z[k] + conj Z[128 - k], t = -i exp(-2 pi i k / 256) (Z[k] - conj Z[128 - k]).
    static_for<0, M / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int ib = Q ? M - 1 - i : (M - i) % M;
      const float2 Bc = cconj(a[ib]);
      const float2 e2 = cadd(a[i], Bc);
      const float2 t2 = twiddle<-1, W, 2 * i + Q>(rot90<-1>(csub(a[i], Bc)));
      r1[i] = cadd(e2, t2);
      r2[i] = cconj(csub(e2, t2));
    });
    if constexpr (Q == 0) {
      const float2 Bc = cconj(a[M / 2]);
      mid = cadd(cadd(a[M / 2], Bc), twiddle<-1, W, M>(rot90<-1>(csub(a[M / 2], Bc))));
    }
  };
  if (odd) r2c(std::integral_constant<int, 1>{});
  else r2c(std::integral_constant<int, 0>{});
  __syncthreads();  // every row of g has been read; the slab now takes X[y][k]
  {
    float2* xrow = slab + y * NC;
    float2* lo = xrow + q;         // k = 2i + q
    float2* hi = xrow + (NC - q);  // 128 - k
    if (odd) {
      lo[0] = r1[0];
      hi[0] = r2[0];
    } else {
      xrow[0] = make_float2(r1[0].x, r2[0].x);  // Gr2[0] + i Gr2[128] (both real)
      xrow[M] = mid;
    }
    static_for<1, M / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      lo[2 * i] = r1[i];
      hi[-2 * i] = r2[i];
    });
  }
  __syncthreads();

  // ------------------------------------------------------------ column DFT (lane (c, h))
  // G[4m + h] = sum_{y'} [sum_j col[y' + 64 j] (-i)^{h j}] exp(-2 pi i h y' / 256) w64^{m y'}
  const int h = __builtin_amdgcn_readfirstlane(l >> 7), c = l & (NC - 1);  // h uniform per wavefront
  float2 Gk[M];
  {
    const float2* col = slab + c;  // column c (c = 0: packed with column 128)
    auto stage = [&](auto hh) {
      constexpr int H = decltype(hh)::value;
      static_for<0, M>([&](auto yy) {
        constexpr int yq = decltype(yy)::value;
        float2 s = col[yq * NC];
        static_for<1, 4>([&](auto jj) {
          constexpr int j = decltype(jj)::value;
          s = cadd(s, twiddle<-1, 4, H * j>(col[(yq + 64 * j) * NC]));
        });
        Gk[yq] = twiddle<-1, W, H * yq>(s);
        if constexpr (yq % 8 == 7) __builtin_amdgcn_sched_barrier(0);
      });
    };
    switch (h) {
      case 0: stage(std::integral_constant<int, 0>{}); break;
      case 1: stage(std::integral_constant<int, 1>{}); break;
      case 2: stage(std::integral_constant<int, 2>{}); break;
      default: stage(std::integral_constant<int, 3>{}); break;
    }
    fft<M, -1>(Gk);
  }
  if (c == 0) {
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      s_nyq[D * m + h] = Gk[m];
    });
  }
  // phase tables (lanes 0..255: one row each)
  const float nu = (float)c * (1.f / W);
  const float hW = (float)h * (1.f / W);
  float sx, cx;
  sincospi_poly(-2.f * G.fx * nu, &sx, &cx);
  const bool nyq_lane = l < W;
  const float omN = (l < W / 2) ? (float)l * (1.f / W) : (l == W / 2 ? 0.5f : (float)(l - W) * (1.f / W));
  float sy = 0.f, cy = 1.f, sxh, cxh;
  sincospi_poly(-G.fx, &sxh, &cxh);
  if (nyq_lane) {
    sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
    s_py[l] = make_float2(cy, sy);
    if (l == W / 2) s_py[W] = make_float2(cy, -sy);  // omega = -1/2: conjugate of omega = +1/2
  }
  __syncthreads();
  float2 GN = make_float2(0.f, 0.f);
  if (nyq_lane) {
    const float2 za = s_nyq[l], zb = cconj(s_nyq[(W - l) & (W - 1)]);
    const float2 d = csub(za, zb);
    GN = make_float2(0.5f * d.y, -0.5f * d.x);
  }
  if (c == 0) {
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 zb = cconj(s_nyq[(W - D * m - h) & (W - 1)]);
      Gk[m] = cscale(cadd(Gk[m], zb), 0.5f);
    });
  }

  // ------------------------------------------------------------ points and U0
  float ure[NP], uim[NP];
  auto point = [&](auto jj, float& n_, float& o_) {
    constexpr int j = decltype(jj)::value;
    if constexpr (j < M) {
      n_ = nu;
      if constexpr (D * j < W / 2) o_ = (float)(D * j) * (1.f / W) + hW;
      else if constexpr (D * j == W / 2) o_ = h ? (float)(W / 2 - W) * (1.f / W) + hW : 0.5f;
      else o_ = (float)(D * j - W) * (1.f / W) + hW;
    } else if constexpr (j == M) {
      n_ = nu;
      o_ = -0.5f;
    } else {
      n_ = (j - M) & 1 ? 0.5f : -0.5f;
      o_ = omN;
    }
  };
  {
    const float colw = (c == 0 ? 0.5f : 1.f) / ((float)W * (float)W);
    const float2 px = make_float2(cx, sx);
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      const float2 P = p.psf_main[m * (D * NC) + D * c + h];
      const float2 gp2 = cmul(cscale(cmulc(P, Gk[m]), colw), px);
      float2 u;
      if constexpr (D * m == W / 2) {
        const float2 q0 = s_py[W / 2 + h];
        const float2 pyA = h ? q0 : cscale(q0, 0.5f);
        u = cmul(gp2, pyA);
        const float2 pyB = h ? make_float2(0.f, 0.f) : cscale(s_py[W], 0.5f);
        const float2 ux = cmul(gp2, pyB);
        ure[M] = ux.x;
        uim[M] = ux.y;
      } else {
        u = cmul(gp2, s_py[D * m + h]);
      }
      ure[m] = u.x;
      uim[m] = u.y;
    });
    const float2 gamN = nyq_lane ? cscale(cmulc(p.psf_nyq[l], GN), 0.25f / ((float)W * (float)W))
                                 : make_float2(0.f, 0.f);
    const bool corner = (l == W / 2);
    const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
    const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
    const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
    const float2 u1 = cmul(cmul(gamN, eM), pyA), u2 = cmul(cmul(gamN, eP), pyA);
    const float2 u3 = cmul(cmul(gamN, eM), pyB), u4 = cmul(cmul(gamN, eP), pyB);
    // corner twins folded into their partners (the transform is even; see the
    // W <= 128 adjoint)
    ure[M + 1] = u1.x + u4.x; uim[M + 1] = u1.y - u4.y;
    ure[M + 2] = u2.x + u3.x; uim[M + 2] = u2.y - u3.y;
  }

  // ------------------------------------------------------------ component loop
  float ax = 0.f, ay = 0.f, a11 = 0.f, a12 = 0.f, a22 = 0.f;
  float* s_pk = s_tile;  // [kKmax][BLOCK] per-lane p_k partials (the tile is no longer needed)
  for (int k = 0; k < kKmax; ++k) s_pk[k * BLOCK + l] = 0.f;
  static_for<0, (NP + PB - 1) / PB>([&](auto bb) {
    constexpr int b0 = decltype(bb)::value * PB;
    constexpr int nb = (NP - b0) < PB ? (NP - b0) : PB;
    float gq[nb], S[nb], S1[nb];
    static_for<0, nb>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      float n_, o_;
      point(std::integral_constant<int, b0 + j>{}, n_, o_);
      gq[j] = kQ * fmaf(G.b11 * n_, n_, fmaf(2.f * G.b12 * n_, o_, G.b22 * o_ * o_));
    });
    {  // component 0 initialises the sums (as in the W <= 128 adjoint)
      const float4 cp = s_cmp[0];
      const float v = cp.x, wa = cp.y, wav = cp.z;
      float pk = 0.f;
      static_for<0, nb>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const float e = __builtin_amdgcn_exp2f(v * gq[j]);
        S[j] = wa * e;
        S1[j] = wav * e;
        pk = fmaf(ure[b0 + j], e, pk);
      });
      s_pk[l] += pk;
    }
    // the next component's constants read one iteration ahead (clamped into
    // the table; the last read is not used), two components per trip
    float4 cpn = s_cmp[1];
#pragma unroll 2
    for (int k = 1; k < G.K; ++k) {
      const float4 cp = cpn;
      cpn = s_cmp[min(k + 1, kKmax - 1)];
      if (cp.w == 0.f) continue;  // A_k = 0 still needs p_k for dL/dA_k
      const float v = cp.x, wa = cp.y, wav = cp.z;
      float pk = 0.f;
      static_for<0, nb>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const float e = __builtin_amdgcn_exp2f(v * gq[j]);
        S[j] = fmaf(wa, e, S[j]);
        S1[j] = fmaf(wav, e, S1[j]);
        pk = fmaf(ure[b0 + j], e, pk);
      });
      s_pk[k * BLOCK + l] += pk;
    }
    static_for<0, nb>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      float n_, o_;
      point(std::integral_constant<int, b0 + j>{}, n_, o_);
      const float si = S[j] * uim[b0 + j];
      const float r1 = S1[j] * ure[b0 + j];
      ax = fmaf(n_, si, ax);
      ay = fmaf(o_, si, ay);
      a11 = fmaf(n_ * n_, r1, a11);
      a12 = fmaf(n_ * o_, r1, a12);
      a22 = fmaf(o_ * o_, r1, a22);
    });
    // Materialise the block's contribution here, so the compiler does not sink
    // the accumulation (and keep this block's sums alive) past later blocks.
    asm volatile("" : "+v"(ax), "+v"(ay), "+v"(a11), "+v"(a12), "+v"(a22));
  });
  ax = block_sum512(ax, s_red);
  ay = block_sum512(ay, s_red);
  a11 = block_sum512(a11, s_red);
  a12 = block_sum512(a12, s_red);
  a22 = block_sum512(a22, s_red);
  // p_k: wavefront sums, then the 8 wavefronts in order
  for (int k = 0; k < G.K; ++k) {
    float v = s_pk[k * BLOCK + l];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    if ((l & 63) == 0) s_pkw[k][wv] = v;
  }
  __syncthreads();
  if (l < G.K) {
    float acc = 0.f;
    for (int w = 0; w < NWAVE; ++w) acc += s_pkw[l][w];
    s_pkw[l][0] = acc;
  }
  __syncthreads();
  if (wv == 0) {  // lanes 0..15 take one component each; lane 0 finishes
    Galaxy Gc = load_galaxy<W>(p, gidx);  // reloaded: keeps G's registers free in the loop above
    make_uniform(Gc);
    CompTerms t = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (l < kKmax)
      t = bwd_component_terms<W>(p, Gc, l, rmask, &s_pkw[0][0], NWAVE, &s_racc[0][0], amp_part + gidx * kKmax);
    t = sum16(t);
    if (l == 0) bwd_chain_finish<W>(p, Gc, gidx, ax, ay, a11, a12, a22, t, grad_params);
  }
}

hipError_t launch_bwd_w256(const RenderArgs& args, const float* gout, float* grad_params, float* amp_part,
                           hipStream_t stream) {
  using namespace bigb;
  constexpr int64_t kChunk = 1024;
  const int64_t nb = std::min<int64_t>(args.n, kChunk);
  float2* scratch = nullptr;
  hipError_t e = hipMallocAsync((void**)&scratch, (size_t)nb * SLAB * sizeof(float2), stream);
  if (e != hipSuccess) return e;
  RenderArgs p = args;
  for (int64_t done = 0; done < args.n; done += kChunk) {
    const int64_t chunk = std::min<int64_t>(args.n - done, kChunk);
    p.x = args.x + done;
    p.y = args.y + done;
    p.flux = args.flux + done;
    p.r_e = args.r_e + done;
    p.e1 = args.e1 + done;
    p.e2 = args.e2 + done;
    p.mix_id = args.mix_id ? args.mix_id + done : nullptr;
    p.n = chunk;
    hipLaunchKernelGGL(render_bwd_w256_kernel, dim3((unsigned)chunk), dim3(BLOCK), 0, stream, p,
                       gout + done * (int64_t)W * W, grad_params + done * 6, amp_part + done * kKmax, scratch);
    e = hipGetLastError();
    if (e != hipSuccess) break;
  }
  hipError_t e2 = hipFreeAsync(scratch, stream);
  return e != hipSuccess ? e : e2;
}

}  // namespace gfc
