// Forward render kernel for 256 x 256 stamps (Lang 2020, Section 2, steps 3-8).
//
// The half spectrum of a 256^2 stamp (257 KB as complex float32) exceeds the
// 160 KB of LDS of a CU, so a 512-thread workgroup renders a stamp in four
// phases and parks the column-transformed spectrum in a device scratch slab.
// One workgroup fits per CU, so the launch is persistent: one workgroup per
// CU takes stamps in turn and reuses its slab while it is in L2 / the MALL.
// A stamp's phases:
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
//                row transform, the integer roll of the centre and the
//                real-space components (step 8), then coalesced stores.
#include "gfc_device.hpp"
#include "gfc_launch.hpp"

namespace gfc {

namespace big {
constexpr int W = 256;
constexpr int D = 4;             // column-transform decimation
constexpr int M = W / D;         // 64 values per lane in the column phase
constexpr int NC = W / 2;        // 128 regular columns
constexpr int BLOCK = NC * D;    // 512 threads
constexpr int CCH = 32;          // columns per combine chunk
constexpr int RCH = 64;          // rows per store chunk
constexpr int SLAB = (NC + 1) * W;  // float2 per stamp in the scratch slab
// LDS: combine chunk = CCH*D*M float2 = 64 KB; store chunk = 2 halves x RCH x 64 float2 = 64 KB
constexpr int LDS_F2 = CCH * D * M;
static_assert(LDS_F2 == 2 * RCH * (W / 4), "shared buffer sizes differ");
}  // namespace big

// EIG: spatially varying PSF (eigen-PSF components with polynomial weights).
template <bool EIG>
__global__ void __launch_bounds__(big::BLOCK)
render_w256_kernel(RenderArgs p, float2* __restrict__ scratch) {
  using namespace big;
  __shared__ float2 s_buf[LDS_F2];
  __shared__ float2 s_py[W + 2];
  __shared__ float2 s_nyq[W];
  __shared__ float2 s_rs[kKmax];  // (v, (1 - w) A) of the components with a real-space share
  __shared__ float s_cj[kEigMax];  // eigen-PSF component weights at this galaxy's position

  // Persistent workgroups: one per CU, each with its own slab, which the
  // next stamp reuses while it is still in L2 / the MALL.
  float2* slab = scratch + (int64_t)blockIdx.x * SLAB;
  for (int64_t stamp = blockIdx.x; stamp < p.n; stamp += gridDim.x) {
    // The lane index is renewed opaquely each stamp, so lane-dependent values
    // are recomputed per stamp instead of being held across the whole loop.
    int l = threadIdx.x;
    asm volatile("" : "+v"(l));
    Galaxy G = load_galaxy<W>(p, stamp);
    make_uniform(G);
    const float* amp = p.amp + G.table * kKmax;
    const float* var = p.var + G.table * kKmax;
    const float trB = G.b11 + G.b22;

    // ---------------------------------------------------------------- column phase
    const int c = l >> 2, h = l & 3;
    const float nu = (float)c * (1.f / W);
    const float hW = (float)h * (1.f / W);
    const float g0 = kQ * G.b11 * nu * nu;
    const float g1 = 2.f * kQ * G.b12 * nu;
    const float g2 = kQ * G.b22;
    float qv[M + 1];
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      float om;
      if constexpr (D * m < W / 2) om = (float)(D * m) * (1.f / W) + hW;
      else if constexpr (D * m == W / 2) om = h ? (float)(W / 2 - W) * (1.f / W) + hW : 0.5f;
      else om = (float)(D * m - W) * (1.f / W) + hW;
      qv[m] = fmaf(om, fmaf(g2, om, g1), g0);
    });
    qv[M] = fmaf(-0.5f, fmaf(g2, -0.5f, g1), g0);  // Nyquist row, omega = -1/2

    const bool nyq_lane = l < W;  // lanes 0..255 also take one row of column k_x = 128
    const float omN = (l < W / 2) ? (float)l * (1.f / W) : (l == W / 2 ? 0.5f : (float)(l - W) * (1.f / W));
    const float qa = kQ * G.b11 * 0.25f, qb = kQ * G.b12, qd = kQ * G.b22;
    // (+1/2, omN) and (-1/2, omN).  The corner's omega = -1/2 twins equal
    // the (-+1/2, +1/2) pair of lane W/2: the mixture transform is even.
    float qn[2];
    qn[0] = fmaf(omN, fmaf(qd, omN, qb), qa);
    qn[1] = fmaf(omN, fmaf(qd, omN, -qb), qa);

    float S[M + 1];
    float SN[2] = {0.f, 0.f};
    static_for<0, M + 1>([&](auto mm) { S[decltype(mm)::value] = 0.f; });
    unsigned rmask = 0;
    for (int k = 0; k < G.K; ++k) {
      const float v = var[k];
      const float A = amp[k];
      const float w = route_weight<W>(v * trB, p.flags);
      if (w < 1.f && A != 0.f) {
        rmask |= 1u << k;
        if (l == 0) s_rs[k] = make_float2(v, (1.f - w) * A);
      }
      const float wa = w * A;
      if (wa == 0.f) continue;
      static_for<0, M + 1>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        S[m] = fmaf(wa, __builtin_amdgcn_exp2f(v * qv[m]), S[m]);
      });
      if (nyq_lane) {
        static_for<0, 2>([&](auto jj) {
          constexpr int j = decltype(jj)::value;
          SN[j] = fmaf(wa, __builtin_amdgcn_exp2f(v * qn[j]), SN[j]);
        });
      }
    }

    // PSF Gaussian and Nyquist-column PSF value (step 2; for a varying PSF the
    // weighted sums of the components' moments and transforms).
    float pg[6];
    float2 psfN = make_float2(0.f, 0.f);
    if constexpr (EIG) {
      const float u = uniform_f((p.psf_px[stamp] - p.eig_norm[0]) * p.eig_norm[1]);
      const float v = uniform_f((p.psf_py[stamp] - p.eig_norm[2]) * p.eig_norm[3]);
      const float up[4] = {1.f, u, u * u, u * u * u}, vp[4] = {1.f, v, v * v, v * v * v};
      if (l < p.eig_J) s_cj[l] = eigen_weight(p, l, up, vp);
      __syncthreads();
      float mom[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int j = 0; j < p.eig_J; ++j) {
        const float cj = s_cj[j];
        static_for<0, 6>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          mom[i] = fmaf(cj, p.eig_mom[j * 6 + i], mom[i]);
        });
        if (nyq_lane) {
          const float2 qn = p.psf_nyq[j * p.eig_stride + l];
          psfN = make_float2(fmaf(cj, qn.x, psfN.x), fmaf(cj, qn.y, psfN.y));
        }
      }
      eigen_gauss(mom, pg);
    } else {
      static_for<0, 6>([&](auto ii) { pg[decltype(ii)::value] = p.pg[decltype(ii)::value]; });
      if (nyq_lane) psfN = p.psf_nyq[l];
    }

    float sx, cx;
    sincospi_poly(-2.f * G.fx * nu, &sx, &cx);
    const float fs = G.flux * (1.f / ((float)W * (float)W));
    const float2 pxF = make_float2(fs * cx, fs * sx);
    if (nyq_lane) {
      float sy, cy, sxh, cxh;
      sincospi_poly(-2.f * G.fy * omN, &sy, &cy);
      sincospi_poly(-G.fx, &sxh, &cxh);
      s_py[l] = make_float2(cy, sy);
      if (l == W / 2) s_py[W] = make_float2(cy, -sy);  // omega = -1/2: conjugate of omega = +1/2
      const float2 eM = make_float2(cxh, sxh), eP = make_float2(cxh, -sxh);
      const bool corner = (l == W / 2);
      const float2 pyA = corner ? make_float2(0.5f * cy, 0.5f * sy) : make_float2(cy, sy);
      const float2 pyB = corner ? make_float2(0.5f * cy, -0.5f * sy) : make_float2(0.f, 0.f);
      const float2 plus = cadd(cscale(pyA, SN[0]), cscale(pyB, SN[1]));
      const float2 minus = cadd(cscale(pyA, SN[1]), cscale(pyB, SN[0]));
      s_nyq[l] = cmul(cscale(psfN, 0.5f * fs), cadd(cmul(eM, plus), cmul(eP, minus)));
    }
    __syncthreads();

    float2 Z[M];
    static_for<0, M>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      float2 P;
      if constexpr (EIG) {
        P = make_float2(0.f, 0.f);
        for (int j = 0; j < p.eig_J; ++j) {
          const float cj = s_cj[j];
          const float2 q = p.psf_main[j * p.eig_stride + m * BLOCK + l];
          P = make_float2(fmaf(cj, q.x, P.x), fmaf(cj, q.y, P.y));
        }
      } else {
        P = p.psf_main[m * BLOCK + l];
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
    if (c == 0) {
      static_for<0, M>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        const float2 xn = s_nyq[D * m + h];
        Z[m] = make_float2(Z[m].x - xn.y, Z[m].y + xn.x);
      });
    }
    fft<M, +1>(Z);

    // ---------------------------------------------------------------- combine
    // X_c[j + 64 q] = sum_h i^{h q} w^{h j} E_{h,c}[j],  w = exp(2 pi i / 256):
    // one radix-4 butterfly per (column, j) gives the four rows j + 64 q.
    // Lane j of wavefront wv takes columns wv, wv + 8, wv + 16, wv + 24 of the chunk.
    {
      const int j = l & (M - 1), wv = l >> 6;
      const float2 w1 = twiddle_rt<+1, W>(j), w2 = twiddle_rt<+1, W>(2 * j), w3 = twiddle_rt<+1, W>(3 * j);
      for (int t = 0; t < NC / CCH; ++t) {
        if ((c / CCH) == t) {
          const int base = ((c % CCH) * D + h) * M;
          static_for<0, M>([&](auto jj) {
            constexpr int jx = decltype(jj)::value;
            s_buf[base + jx] = Z[jx];
          });
        }
        __syncthreads();
        static_for<0, CCH / (BLOCK / M)>([&](auto bb) {
          constexpr int b = decltype(bb)::value;
          const int cl = wv + b * (BLOCK / M);
          const float2* e = &s_buf[(cl * D) * M + j];
          const float2 t0 = e[0], t1 = cmul(w1, e[M]), t2 = cmul(w2, e[2 * M]), t3 = cmul(w3, e[3 * M]);
          const float2 a = cadd(t0, t2), bq = csub(t0, t2), cq = cadd(t1, t3), d = rot90<+1>(csub(t1, t3));
          const float2 x0 = cadd(a, cq), x1 = cadd(bq, d), x2 = csub(a, cq), x3 = csub(bq, d);
          const int cg = t * CCH + cl;
          if (cg == 0) {  // column 0 carries column 128 as its imaginary part
            slab[j] = make_float2(x0.x, 0.f);
            slab[j + 64] = make_float2(x1.x, 0.f);
            slab[j + 128] = make_float2(x2.x, 0.f);
            slab[j + 192] = make_float2(x3.x, 0.f);
            slab[NC * W + j] = make_float2(x0.y, 0.f);
            slab[NC * W + j + 64] = make_float2(x1.y, 0.f);
            slab[NC * W + j + 128] = make_float2(x2.y, 0.f);
            slab[NC * W + j + 192] = make_float2(x3.y, 0.f);
          } else {
            float2* o = slab + cg * W + j;
            o[0] = x0;
            o[64] = x1;
            o[128] = x2;
            o[192] = x3;
          }
        });
        __syncthreads();
      }
    }

    // ---------------------------------------------------------------- row phase
    // Wavefront wv = l / 64 takes rows 64 (wv / 2) .. +63 and the half q = wv % 2
    // of the complex-to-real transform: R[k] for k = 2i + q.
    const int wv = l >> 6;
    const int q = wv & 1;
    const int y = ((wv >> 1) << 6) | (l & 63);
    float2 Rq[M];
    if (q == 0) {
      // pairs (k, 128 - k) with k = 2i: indices i and 64 - i of X[2i]
      float2 Xe[M + 1];
      static_for<0, M + 1>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        Xe[i] = slab[(2 * i) * W + y];
      });
      static_for<0, M / 2 + 1>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        constexpr int k = 2 * i;
        const float2 a = Xe[i], b = cconj(Xe[M - i]);
        const float2 sum = cadd(a, b);
        const float2 tt = twiddle<+1, W, k>(csub(a, b));
        Rq[i] = make_float2(sum.x - tt.y, sum.y + tt.x);
        if constexpr (i != 0 && 2 * i != M) Rq[M - i] = make_float2(sum.x + tt.y, tt.x - sum.y);
      });
    } else {
      // pairs (k, 128 - k) with k = 2i + 1: indices i and 63 - i of X[2i + 1]
      float2 Xo[M];
      static_for<0, M>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        Xo[i] = slab[(2 * i + 1) * W + y];
      });
      static_for<0, M / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        constexpr int k = 2 * i + 1;
        const float2 a = Xo[i], b = cconj(Xo[M - 1 - i]);
        const float2 sum = cadd(a, b);
        const float2 tt = twiddle<+1, W, k>(csub(a, b));
        Rq[i] = make_float2(sum.x - tt.y, sum.y + tt.x);
        Rq[M - 1 - i] = make_float2(sum.x + tt.y, tt.x - sum.y);
      });
    }
    fft<M, +1>(Rq);  // z_q[n] = sum_i R[2i + q] w64^{i n}

    // ---------------------------------------------------------------- store
    // z[n] = z_0[n mod 64] + s w128^{n mod 64} z_1[n mod 64], s = +1 (n < 64) or -1;
    // pixel x of the fractional image row is Re z[x/2] (x even) or Im z[x/2].
    const int X = l & (W - 1), rh = l >> 8;
    const int xs = (X - G.nx) & (W - 1);
    const int n = xs >> 1, nn = n & (M - 1);
    const float2 tw = twiddle_rt<+1, 2 * M>(nn);
    const float sg = (n < M) ? 1.f : -1.f;
    // value = z0.part + sg * (ca * z1.x + cb * z1.y)
    const bool odd = xs & 1;
    const float ca = sg * (odd ? tw.y : tw.x);
    const float cb = sg * (odd ? tw.x : -tw.y);
    const float dx = (float)X - G.x0 - pg[0];
    float* outp = p.out + stamp * (int64_t)(W * W);
    for (int t = 0; t < W / RCH; ++t) {
      if ((wv >> 1) == t) {
        // tile [q][row - 64 t][n]
        float2* dst = &s_buf[(q * RCH + (y - t * RCH)) * M];
        static_for<0, M>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          dst[i] = Rq[i];
        });
      }
      __syncthreads();
      constexpr int RPL = RCH / 2;  // rows per lane in this chunk
      float val[RPL];
      const float* tile = reinterpret_cast<const float*>(s_buf);
      static_for<0, RPL>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        const int srow = rh * RPL + r;
        const float z0 = tile[2 * (srow * M + nn) + (odd ? 1 : 0)];
        const float2 z1 = s_buf[(RCH + srow) * M + nn];
        val[r] = fmaf(ca, z1.x, fmaf(cb, z1.y, z0));
      });
      const int srow0 = t * RCH + rh * RPL;
      for (unsigned mk = rmask; mk != 0; mk &= mk - 1) {
        const float2 rs = s_rs[__builtin_ctz(mk)];  // LDS, not global: no wait on the stores above
        const float v = rs.x, ra = rs.y;
        const float sxx = fmaf(v, G.b11, pg[2]);
        const float sxy = fmaf(v, G.b12, pg[3]);
        const float syy = fmaf(v, G.b22, pg[4]);
        const float det = fmaf(sxx, syy, -(sxy * sxy));
        const float rdet = __builtin_amdgcn_rcpf(det);
        const float ampr = ra * G.flux * pg[5] * kInv2Pi * __builtin_amdgcn_rsqf(det);
        const float a0 = kHalfLog2e * (syy * rdet) * dx * dx;
        const float a1 = -2.f * kHalfLog2e * (sxy * rdet) * dx;
        const float a2 = kHalfLog2e * (sxx * rdet);
        static_for<0, RPL>([&](auto rr) {
          constexpr int r = decltype(rr)::value;
          const int Y = (srow0 + r + G.ny) & (W - 1);
          const float dy = (float)Y - G.y0 - pg[1];
          val[r] = fmaf(ampr, __builtin_amdgcn_exp2f(fmaf(dy, fmaf(a2, dy, a1), a0)), val[r]);
        });
      }
      static_for<0, RPL>([&](auto rr) {
        constexpr int r = decltype(rr)::value;
        const int Y = (srow0 + r + G.ny) & (W - 1);
        const float v = (p.flags & kAccumulate) ? val[r] + outp[Y * W + X] : val[r];
        __builtin_nontemporal_store(v, &outp[Y * W + X]);  // streamed output
      });
      __syncthreads();
    }
    if (!G.ok && l == 0) atomicAdd(p.invalid, 1ull);
  }  // stamps of this workgroup (the store loop ends with a barrier)
}

hipError_t launch_render_w256(const RenderArgs& args, hipStream_t stream) {
  using namespace big;
  // One workgroup per CU (the kernel's registers allow one 512-thread
  // workgroup per CU), so the slabs in use total CUs x 264 KB.
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int64_t nb = std::min<int64_t>(args.n, std::max(cus, 1));
  float2* scratch = nullptr;
  e = hipMallocAsync((void**)&scratch, (size_t)nb * SLAB * sizeof(float2), stream);
  if (e != hipSuccess) return e;
  if (args.eig_J > 0)
    hipLaunchKernelGGL(render_w256_kernel<true>, dim3((unsigned)nb), dim3(BLOCK), 0, stream, args, scratch);
  else
    hipLaunchKernelGGL(render_w256_kernel<false>, dim3((unsigned)nb), dim3(BLOCK), 0, stream, args, scratch);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(scratch, stream);
  return e != hipSuccess ? e : e2;
}

}  // namespace gfc
