// Forward render kernel for 256 x 256 stamps (Lang 2020, Section 2, steps 3-8).
//
// The half spectrum of a 256^2 stamp (257 KB as complex float32) exceeds the
// 160 KB of LDS of a CU, so a workgroup renders a stamp in four phases and
// parks the column-transformed spectrum in a device scratch slab.  A
// workgroup has 256 threads and takes each phase's 512 work items in two
// rounds, so two independent workgroups share a CU (one's barriers and
// memory waits overlap the other's arithmetic).  The launch is persistent:
// the resident workgroups take stamps in turn and each reuses its slab while
// it is in L2 / the MALL.  A stamp's phases:
//
//  column phase  lane (c, h), c = 0..127, h = 0..3, evaluates the mixture
//                transform on column k_x = c, rows k_y = 4m + h (steps 5-6),
//                applies phase, flux and PSF spectrum (step 7a) and runs a
//                64-point inverse FFT in registers.  Column k_x = 128 is packed
//                into column 0 as its imaginary part.
//  combine       the last radix-4 stage of the 256-point column transform, 32
//                columns at a time through LDS; results go to the slab,
//                column-major.
//  row phase     wavefronts alternate between the even and odd half of the
//                complex-to-real row transform (a 128-point complex FFT split
//                into two 64-point FFTs); the split is uniform per wavefront.
//  store         64 rows at a time through LDS: the last radix-2 stage of the
//                row transform, the integer roll of the x centre (the integer
//                y shift is a phase in the y-phase table, so rows arrive in
//                output order) and the real-space components (step 8), then
//                coalesced stores.
#include "gfc_device.hpp"
#include "gfc_launch.hpp"

namespace gfc {

template <int W_>
struct LargeCfg {
  static constexpr int W = W_;
  static constexpr int D = 4;             // column-transform decimation
  static constexpr int M = W / D;         // values per item in the column phase
  static constexpr int NC = W / 2;        // regular columns
  static constexpr int NL = NC * D;       // (column, h) items
  static constexpr int BLOCK = 256;       // threads per workgroup
  static constexpr int NR = NL / BLOCK;   // rounds per phase (1 at 128, 2 at 256)
  static constexpr int CCH = 32;          // columns per combine chunk
  static constexpr int RCH = 64;          // rows per store chunk
  static constexpr int RPL = 32;          // rows a thread finishes per pass over a store chunk
  static constexpr int XPT = BLOCK / W;   // threads per output column in the store (1 or 2)
  static constexpr int PASSES = RCH / (RPL * XPT);
  static constexpr int SLAB = (NC + 1) * W;  // float2 per stamp in the scratch slab
  // Rows of M float2 are M + 1 apart in LDS: a wavefront's lanes each write
  // their own row, and an odd stride puts those rows in different banks.
  static constexpr int MP = M + 1;
  // LDS: combine chunk = CCH*D rows; store chunk = 2 halves x RCH rows
  static constexpr int LDS_F2 = CCH * D * MP;
  static_assert(LDS_F2 == 2 * RCH * MP, "shared buffer sizes differ");
  static_assert(W == 128 || W == 256, "stamp sizes 128 and 256");
  static_assert(XPT * W == BLOCK && NR * BLOCK == NL, "thread counts");
  static_assert((NC / CCH) == 2 * NR && (W / RCH) == 2 * NR, "two combine and two store chunks per round");
};

// Index of bin (column c, row k_y) in the cached PSF spectrum: at 256 the
// cache is in this kernel's item order (l = 4c + h, rows 4m + h); at 128 it is
// in the order of the other 128 x 128 kernels (l = 2c + h', rows 2m' + h').
template <int W>
__device__ __forceinline__ int psf_index(int m, int l) {
  if constexpr (W == 256) {
    return m * (2 * W) + l;
  } else {
    const int c = l >> 2, h = l & 3;
    return (2 * m + (h >> 1)) * W + 2 * c + (h & 1);
  }
}

// EIG: spatially varying PSF (eigen-PSF components with polynomial weights).
// PT: each galaxy names its constant PSF in p.psf_id (serving batches mix PSFs).
template <int W, bool EIG, bool PT>
__global__ void __launch_bounds__(LargeCfg<W>::BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
render_large_kernel(RenderArgs p, float2* __restrict__ scratch) {
  using C = LargeCfg<W>;
  constexpr int D = C::D, M = C::M, MP = C::MP, NC = C::NC, NL = C::NL, BLOCK = C::BLOCK, NR = C::NR,
                CCH = C::CCH, RCH = C::RCH, RPL = C::RPL, SLAB = C::SLAB, LDS_F2 = C::LDS_F2;
  __shared__ float2 s_buf[LDS_F2];
  __shared__ float2 s_py[W + 2];
  __shared__ float2 s_nyq[W];
  __shared__ float2 s_rs[kKmax];  // (v, (1 - w) A) of the components with a real-space share
  __shared__ float s_cj[kEigMax];  // eigen-PSF component weights at this galaxy's position

  float2* slab = scratch + (int64_t)blockIdx.x * SLAB;
  for (int64_t stamp = blockIdx.x; stamp < p.n; stamp += gridDim.x) {
    // The thread index is renewed opaquely each stamp, so thread-dependent
    // values are recomputed per stamp instead of being held across the loop.
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    Galaxy G = load_galaxy<W>(p, stamp);
    make_uniform(G);
    const float2* psfm = p.psf_main;
    const float2* psfn = p.psf_nyq;
    int ps = 0;
    if constexpr (PT) {
      static_assert(!EIG, "a per-galaxy PSF index takes constant PSFs");
      ps = __builtin_amdgcn_readfirstlane(p.psf_id[stamp]);
      if (ps < 0 || ps >= p.n_psf) {  // invalid galaxy: NaN stamp, counted
        ps = 0;
        G.ok = false;
        G.flux = __builtin_nanf("");
      }
      psfm = p.psf_main_tab[ps];
      psfn = p.psf_nyq_tab[ps];
    }
    const float* amp = p.amp + G.table * kKmax;
    const float* var = p.var + G.table * kKmax;
    const float trB = G.b11 + G.b22;
    const float fs = G.flux * (1.f / ((float)W * (float)W));

    // PSF Gaussian (step 2; for a varying PSF the weighted sums of the
    // components' moments).
    float pg[6];
    if constexpr (EIG) {
      const float u = uniform_f((p.psf_px[stamp] - p.eig_norm[0]) * p.eig_norm[1]);
      const float v = uniform_f((p.psf_py[stamp] - p.eig_norm[2]) * p.eig_norm[3]);
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
    } else if constexpr (PT) {
      static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg_tab[6 * ps + decltype(ii)::value]; });
    } else {
      static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg[decltype(ii)::value]; });
    }

    // ------------------------------------------------------------ column phase + combine
    // Round rd takes items l = t + 256 rd: column c = l / 4 (0..63, then
    // 64..127), rows k_y = 4m + h, and the combine chunks of its columns.
    unsigned rmask = 0;
    static_for<0, NR>([&](auto rdd) {
      constexpr int rd = decltype(rdd)::value;
      // renewed per round: nothing thread-dependent is carried between rounds
      int t = threadIdx.x;
      asm volatile("" : "+v"(t));
      const int l = t + rd * BLOCK;
      const int c = l >> 2, h = l & 3;
      const float nu = (float)c * (1.f / W);
      const float hW = (float)h * (1.f / W);
      const float g0 = kQ * G.b11 * nu * nu;
      const float g1 = 2.f * kQ * G.b12 * nu;
      const float g2 = kQ * G.b22;
      // omega = c_m + h/W with a compile-time c_m: the quadratic expanded
      // about h/W is two FMAs with an immediate per bin
      const float e0 = fmaf(hW, fmaf(g2, hW, g1), g0);
      const float e1 = fmaf(2.f * g2, hW, g1);
      float qv[M + 1];
      static_for<0, M>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        if constexpr (D * m == W / 2) {
          const float om = h ? (float)(W / 2 - W) * (1.f / W) + hW : 0.5f;
          qv[m] = fmaf(om, fmaf(g2, om, g1), g0);
        } else if constexpr (m == 0) {
          qv[m] = e0;
        } else {
          constexpr float cm = (D * m < W / 2) ? (float)(D * m) * (1.f / W) : (float)(D * m - W) * (1.f / W);
          qv[m] = fmaf(cm, fmaf(cm, g2, e1), e0);
        }
      });
      qv[M] = fmaf(-0.5f, fmaf(g2, -0.5f, g1), g0);  // Nyquist row, omega = -1/2

      // In round 0 thread t < W also takes row t of column k_x = W/2:
      // (+-1/2, omN).  The corner's omega = -1/2 twins equal the (-+1/2, +1/2)
      // pair of row W/2: the mixture transform is even.
      const bool nyq = t < W;
      const float omN = (t < W / 2) ? (float)t * (1.f / W) : (t == W / 2 ? 0.5f : (float)(t - W) * (1.f / W));
      float qn[2];
      if constexpr (rd == 0) {
        const float qa = kQ * G.b11 * 0.25f, qb = kQ * G.b12, qd = kQ * G.b22;
        qn[0] = fmaf(omN, fmaf(qd, omN, qb), qa);
        qn[1] = fmaf(omN, fmaf(qd, omN, -qb), qa);
      }

      float S[M + 1];
      float SN[2] = {0.f, 0.f};
      static_for<0, M + 1>([&](auto mm) { S[decltype(mm)::value] = 0.f; });
      for (int k = 0; k < G.K; ++k) {
        const float v = var[k];
        const float A = amp[k];
        const float w = route_weight<W>(v * trB, p.flags);
        if constexpr (rd == 0) {
          if (w < 1.f && A != 0.f) {
            rmask |= 1u << k;
            if (t == 0) s_rs[k] = make_float2(v, (1.f - w) * A);
          }
        }
        const float wa = w * A;
        if (wa == 0.f) continue;
        static_for<0, M + 1>([&](auto mm) {
          constexpr int m = decltype(mm)::value;
          S[m] = fmaf(wa, __builtin_amdgcn_exp2f(v * qv[m]), S[m]);
        });
        if constexpr (rd == 0) {
          if (nyq) {
            static_for<0, 2>([&](auto jj) {
              constexpr int j = decltype(jj)::value;
              SN[j] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[j]), SN[j]);
            });
          }
        }
      }

      if (rd == 0 && nyq) {
        // y phase of row t, the omega = -1/2 twin (conjugate of row W/2), and
        // the Nyquist column's row t
        float2 psfN;
        if constexpr (EIG) {
          psfN = make_float2(0.f, 0.f);
          for (int j = 0; j < p.eig_J; ++j) {
            const float cj = s_cj[j];
            const float2 qn2 = p.psf_nyq[j * p.eig_stride + t];
            psfN = make_float2(fmaf(cj, qn2.x, psfN.x), fmaf(cj, qn2.y, psfN.y));
          }
        } else {
          psfN = psfn[t];
        }
        float sy, cy, sxh, cxh;
        sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
        {
          // the integer part of the y centre as a phase too (an exact table
          // entry): the stamp leaves the transforms in output row order
          const float2 ti = twiddle_rt<-1, W>(G.ny * t);
          const float c2 = fmaf(cy, ti.x, -(sy * ti.y)), s2 = fmaf(cy, ti.y, sy * ti.x);
          cy = c2;
          sy = s2;
        }
        sincospi_poly(-G.fx, &sxh, &cxh);
        s_py[t] = make_float2(cy, sy);
        if (t == W / 2) s_py[W] = make_float2(cy, -sy);
        const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
        const bool corner = (t == W / 2);
        const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
        const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
        const float2 plus = cadd(cscale(pyA, SN[0]), cscale(pyB, SN[1]));
        const float2 minus = cadd(cscale(pyA, SN[1]), cscale(pyB, SN[0]));
        s_nyq[t] = cmul(cscale(psfN, 0.5f * fs), cadd(cmul(eM, plus), cmul(eP, minus)));
      }
      if constexpr (rd == 0) __syncthreads();

      float sx, cx;
      sincospi_poly(-2.f * G.fx * nu, &sx, &cx);
      const float2 pxF = make_float2(fs * cx, fs * sx);
      float2 Z[M];
      static_for<0, M>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        float2 P;
        if constexpr (EIG) {
          P = make_float2(0.f, 0.f);
          for (int j = 0; j < p.eig_J; ++j) {
            const float cj = s_cj[j];
            const float2 q = p.psf_main[j * p.eig_stride + psf_index<W>(m, l)];
            P = make_float2(fmaf(cj, q.x, P.x), fmaf(cj, q.y, P.y));
          }
        } else {
          P = psfm[psf_index<W>(m, l)];
        }
        if constexpr (D * m == W / 2) {
          const float2 q0 = s_py[W / 2 + h];
          const float2 pyA = h ? q0 : cscale(q0, 0.5f);
          const float2 pyB = h ? make_float2(0.f, 0.f) : cscale(s_py[W], 0.5f);
          Z[m] = cmul(cmul(P, pxF), cadd(cscale(pyA, S[m]), cscale(pyB, S[M])));
        } else {
          Z[m] = cscale(cmul(cmul(P, s_py[D * m + h]), pxF), S[m]);
        }
      });
      if (c == 0) {  // column 0 carries column W/2 as its imaginary part
        static_for<0, M>([&](auto mm) {
          constexpr int m = decltype(mm)::value;
          const float2 xn = s_nyq[D * m + h];
          Z[m] = make_float2(Z[m].x - xn.y, Z[m].y + xn.x);
        });
      }
      fft<M, +1>(Z);

      // Combine: X_c[j + M q] = sum_h i^{h q} w^{h j} E_{h,c}[j],
      // w = exp(2 pi i / W): one radix-4 butterfly per (column, j) gives the
      // four rows j + M q.  Thread t takes j = t mod M and the chunk's
      // columns t / M, t / M + BLOCK / M, ...
      const int j = t & (M - 1), wv = t / M;
      const float2 w1 = twiddle_rt<+1, W>(j), w2 = twiddle_rt<+1, W>(2 * j), w3 = twiddle_rt<+1, W>(3 * j);
      static_for<0, 2>([&](auto tt) {
        constexpr int tc = 2 * rd + decltype(tt)::value;  // chunk: columns 32 tc .. 32 tc + 31
        if ((c / CCH) == tc) {
          const int base = ((c % CCH) * D + h) * MP;
          static_for<0, M>([&](auto jj) {
            constexpr int jx = decltype(jj)::value;
            s_buf[base + jx] = Z[jx];
          });
        }
        __syncthreads();
        static_for<0, CCH / (BLOCK / M)>([&](auto bb) {
          constexpr int b = decltype(bb)::value;
          const int cl = wv + b * (BLOCK / M);
          const float2* e = &s_buf[(cl * D) * MP + j];
          const float2 t0 = e[0], t1 = cmul(w1, e[MP]), t2 = cmul(w2, e[2 * MP]), t3 = cmul(w3, e[3 * MP]);
          const float2 a = cadd(t0, t2), bq = csub(t0, t2), cq = cadd(t1, t3), d = rot90<+1>(csub(t1, t3));
          const float2 x0 = cadd(a, cq), x1 = cadd(bq, d), x2 = csub(a, cq), x3 = csub(bq, d);
          const int cg = tc * CCH + cl;
          if (cg == 0) {
            slab[j] = make_float2(x0.x, 0.f);
            slab[j + M] = make_float2(x1.x, 0.f);
            slab[j + 2 * M] = make_float2(x2.x, 0.f);
            slab[j + 3 * M] = make_float2(x3.x, 0.f);
            slab[NC * W + j] = make_float2(x0.y, 0.f);
            slab[NC * W + j + M] = make_float2(x1.y, 0.f);
            slab[NC * W + j + 2 * M] = make_float2(x2.y, 0.f);
            slab[NC * W + j + 3 * M] = make_float2(x3.y, 0.f);
          } else {
            float2* o = slab + cg * W + j;
            o[0] = x0;
            o[M] = x1;
            o[2 * M] = x2;
            o[3 * M] = x3;
          }
        });
        __syncthreads();
      });
    });

    // ------------------------------------------------------------ row phase + store
    // Round rr takes items l = t + 256 rr: wavefront wl = l / 64 takes rows
    // 64 (wl / 2) .. +63 and the half q = wl % 2 of the complex-to-real
    // transform, R[k] for k = 2i + q; then the store chunks of those rows.
    float* outp = p.out + stamp * (int64_t)(W * W);
    static_for<0, NR>([&](auto rrr) {
      constexpr int rr = decltype(rrr)::value;
      int t = threadIdx.x;
      asm volatile("" : "+v"(t));
      const int l = t + rr * BLOCK;
      const int wl = l >> 6;
      const int q = wl & 1;
      const int y = ((wl >> 1) << 6) | (l & 63);
      float2 Rq[M];
      if (q == 0) {
        // pairs (k, NC - k) with k = 2i: indices i and M - i of X[2i]
        float2 Xe[M + 1];
        static_for<0, M + 1>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          Xe[i] = slab[(2 * i) * W + y];
        });
        static_for<0, M / 2 + 1>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          constexpr int k = 2 * i;
          float2 lo, hi;
          c2r_pair<+1, W, k>(Xe[i], cconj(Xe[M - i]), lo, hi);
          Rq[i] = lo;
          if constexpr (i != 0 && 2 * i != M) Rq[M - i] = hi;
        });
      } else {
        // pairs (k, NC - k) with k = 2i + 1: indices i and M - 1 - i of X[2i + 1]
        float2 Xo[M];
        static_for<0, M>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          Xo[i] = slab[(2 * i + 1) * W + y];
        });
        static_for<0, M / 2>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          constexpr int k = 2 * i + 1;
          c2r_pair<+1, W, k>(Xo[i], cconj(Xo[M - 1 - i]), Rq[i], Rq[M - 1 - i]);
        });
      }
      fft<M, +1>(Rq);  // z_q[n] = sum_i R[2i + q] w_M^{i n}

      static_for<0, 2>([&](auto tt) {
        constexpr int tc = 2 * rr + decltype(tt)::value;  // chunk: rows 64 tc .. 64 tc + 63
        if ((wl >> 1) == tc) {
          // tile [q][row - 64 tc][n]
          float2* dst = &s_buf[(q * RCH + (y - tc * RCH)) * MP];
          static_for<0, M>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            dst[i] = Rq[i];
          });
        }
        __syncthreads();
        const float* tile = reinterpret_cast<const float*>(s_buf);
        // z[n] = z_0[n mod M] + s w_{2M}^{n mod M} z_1[n mod M], s = +1 (n < M)
        // or -1; pixel x of the fractional image row is Re z[x/2] (x even) or
        // Im z[x/2]: value = z0.part + sg * (ca * z1.x + cb * z1.y)
        int tx = threadIdx.x;
        asm volatile("" : "+v"(tx));
        const int X = tx & (W - 1);  // the output column this thread stores
        const int rx = tx / W;       // and its share of the chunk's rows
        const int xs = (X - G.nx) & (W - 1);
        const int n = xs >> 1, nn = n & (M - 1);
        const float2 tw = twiddle_rt<+1, 2 * M>(nn);
        const float sg = (n < M) ? 1.f : -1.f;
        const bool odd = xs & 1;
        const float ca = sg * (odd ? tw.y : tw.x);
        const float cb = sg * (odd ? tw.x : -tw.y);
        const float dx = (float)X - G.x0 - pg[0];
        static_for<0, C::PASSES>([&](auto hh) {
          constexpr int rh = decltype(hh)::value;
          const int srowb = (rh * C::XPT + rx) * RPL;  // first chunk row of this pass
          float val[RPL];
          static_for<0, RPL>([&](auto rq) {
            constexpr int r = decltype(rq)::value;
            const int srow = srowb + r;
            const float z0 = tile[2 * (srow * MP + nn) + (odd ? 1 : 0)];
            const float2 z1 = s_buf[(RCH + srow) * MP + nn];
            val[r] = fmaf(ca, z1.x, fmaf(cb, z1.y, z0));
          });
          const int srow0 = tc * RCH + srowb;
          for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
            const float2 rs = s_rs[__builtin_ctz(mk)];  // LDS, not global: no wait on the stores above
            const float v = rs.x, ra = rs.y;
            const float sxx = fmaf(v, G.b11, pg[2]);
            const float sxy = fmaf(v, G.b12, pg[3]);
            const float syy = fmaf(v, G.b22, pg[4]);
            const float det = fmaf(sxx, syy, -(sxy * sxy));
            const float rdet = __builtin_amdgcn_rcpf(det);
            const float ampr = ra * G.flux * pg[5] * kInv2Pi * __builtin_amdgcn_rsqf(det);
            // output row srow0 + r: along the column the quadratic form is
            // dx^2 / sxx + (sxx / det) (dy - (sxy / sxx) dx)^2, completed about
            // the conditional mean (no large terms cancel near the peak); the
            // exponent is k - u^2 with u = g (r + m), two FMAs with an
            // immediate per pixel
            const float rsxx = __builtin_amdgcn_rcpf(sxx);
            const float g = sqrtf(-kHalfLog2e * sxx * rdet);
            const float k0 = kHalfLog2e * dx * dx * rsxx;
            const float dyq = (float)srow0 - G.y0 - pg[1];
            const float gm = g * fmaf(-sxy * rsxx, dx, dyq);
            static_for<0, RPL / 2>([&](auto rq) {
              constexpr int r = 2 * decltype(rq)::value;
              const float u0 = fmaf(g, (float)r, gm);
              const float u1 = fmaf(g, (float)(r + 1), gm);
              val[r] = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u0, u0, k0)), val[r]);
              val[r + 1] = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(-u1, u1, k0)), val[r + 1]);
            });
          }
          static_for<0, RPL>([&](auto rq) {
            constexpr int r = decltype(rq)::value;
            const int Y = srow0 + r;
            const float v = (p.flags & kAccumulate) ? val[r] + outp[Y * W + X] : val[r];
            __builtin_nontemporal_store(v, &outp[Y * W + X]);  // streamed output
          });
        });
        __syncthreads();
      });
    });
    if (!G.ok && t == 0) atomicAdd(p.invalid, 1ull);
  }  // stamps of this workgroup (the store loop ends with a barrier)
}

// Workgroups of one instantiation that stay resident at once (occupancy per
// CU x CUs), queried once per instantiation.
template <int W, bool EIG, bool PT>
static hipError_t large_resident(int64_t* out) {
  static int64_t cached = 0;
  if (cached == 0) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, render_large_kernel<W, EIG, PT>, LargeCfg<W>::BLOCK, 0);
    if (e != hipSuccess) return e;
    cached = (int64_t)std::max(per, 1) * std::max(cus, 1);
  }
  *out = cached;
  return hipSuccess;
}

template <int W, bool EIG, bool PT>
static hipError_t launch_large(const RenderArgs& args, hipStream_t stream) {
  using C = LargeCfg<W>;
  // As many workgroups as stay resident, each with its own slab.
  int64_t resident = 0;
  hipError_t e = large_resident<W, EIG, PT>(&resident);
  if (e != hipSuccess) return e;
  const int64_t nb = std::min<int64_t>(args.n, resident);
  float2* scratch = nullptr;
  e = hipMallocAsync((void**)&scratch, (size_t)nb * C::SLAB * sizeof(float2), stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((render_large_kernel<W, EIG, PT>), dim3((unsigned)nb), dim3(C::BLOCK), 0, stream, args, scratch);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(scratch, stream);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_render_w256(const RenderArgs& args, hipStream_t stream) {
  if (args.psf_id) return args.eig_J > 0 ? hipErrorInvalidValue : launch_large<256, false, true>(args, stream);
  return args.eig_J > 0 ? launch_large<256, true, false>(args, stream) : launch_large<256, false, false>(args, stream);
}

}  // namespace gfc
