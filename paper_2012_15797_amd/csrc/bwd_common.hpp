// Shared tail of the adjoint kernels: the chain rule from the frequency- and
// pixel-domain sums of one stamp to d loss / d(x, y, flux, log r_e, e1, e2)
// and the per-galaxy amplitude partials (Section 2, steps 3 and 4
// differentiated).
#pragma once

#include "gfc_device.hpp"

namespace gfc {

// Contributions of mixture component k to the chain rule (dx, dy, dF and the
// three entries of dL/dB), and its amplitude partial written to ap[k].
// pk_sum[k * pk_stride]: the component's Fourier sum p_k; racc[6 k + i]: its
// real-space sums (sum g N, g N z_x, g N z_y, g N z_x^2, g N z_x z_y, g N z_y^2).
struct CompTerms {
  float dx, dy, dF, L11, L12, L22;
};

template <int W>
__device__ inline CompTerms bwd_component_terms(const RenderArgs& p, const Galaxy& G, int k, unsigned rmask,
                                                const float* pk_sum, int pk_stride, const float* racc,
                                                float* ap) {
  CompTerms c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (k >= G.K) {
    ap[k] = 0.f;
    return c;
  }
  const float* amp = p.amp + G.table * kKmax;
  const float* var = p.var + G.table * kKmax;
  const float trB = G.b11 + G.b22;
  const float F = G.flux;
  const float pamp = p.pg[5];
  const float v = var[k];
  const float A = amp[k];
  const float tr = v * trB;
  const float w = route_weight<W>(tr, p.flags);
  const float n = (0.5f * (float)W) * __builtin_amdgcn_rsqf(tr);
  const float pk = pk_sum[k * pk_stride];
  float g0 = 0.f;
  if (rmask & (1u << k)) {
    const float* R = racc + 6 * k;
    g0 = R[0];
    const float sxx = fmaf(v, G.b11, p.pg[2]);
    const float sxy = fmaf(v, G.b12, p.pg[3]);
    const float syy = fmaf(v, G.b22, p.pg[4]);
    const float det = fmaf(sxx, syy, -(sxy * sxy));
    const float rdet = __builtin_amdgcn_rcpf(det);  // det > 0: a covariance convolved with the PSF's
    const float ixx = syy * rdet, ixy = -sxy * rdet, iyy = sxx * rdet;
    const float rk = (1.f - w) * F * A * pamp;
    c.dx = rk * R[1];
    c.dy = rk * R[2];
    c.L11 = 0.5f * rk * v * (R[3] - ixx * R[0]);
    c.L12 = rk * v * (R[4] - ixy * R[0]);
    c.L22 = 0.5f * rk * v * (R[5] - iyy * R[0]);
  }
  c.dF = A * (w * pk + (1.f - w) * pamp * g0);
  ap[k] = G.ok ? F * (w * pk + (1.f - w) * pamp * g0) : 0.f;
  // smooth routing: dL/dw_k * dw/dn * dn/d(b11 or b22)
  const float dLdw = F * A * (pk - pamp * g0);
  const float dn = -0.5f * n * __builtin_amdgcn_rcpf(trB);
  const float t = route_slope<W>(n, p.flags) * dLdw * dn;
  c.L11 += t;
  c.L22 += t;
  return c;
}

// Sum of CompTerms over each group of 16 lanes (fixed butterfly order); every
// lane of the group receives the totals.  Called with every lane active.
__device__ __forceinline__ CompTerms sum16(CompTerms c) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    c.dx += __shfl_xor(c.dx, o);
    c.dy += __shfl_xor(c.dy, o);
    c.dF += __shfl_xor(c.dF, o);
    c.L11 += __shfl_xor(c.L11, o);
    c.L12 += __shfl_xor(c.L12, o);
    c.L22 += __shfl_xor(c.L22, o);
  }
  return c;
}

// The rest of the chain rule on one lane: ax, ay, a11, a12, a22 are the stamp
// sums of the Fourier-path terms (see the adjoint kernels), tot the summed
// component terms; B -> C0 -> (log r_e, e1, e2).
template <int W>
__device__ inline void bwd_chain_finish(const RenderArgs& p, const Galaxy& G, int64_t gidx, float ax, float ay,
                                        float a11, float a12, float a22, const CompTerms& tot,
                                        float* grad_params) {
  constexpr float kPi = 3.14159265358979f;
  const float F = G.flux;
  const float dxs = fmaf(2.f * kPi * F, ax, tot.dx);
  const float dys = fmaf(2.f * kPi * F, ay, tot.dy);
  const float L11 = fmaf(-2.f * kPi * kPi * F, a11, tot.L11);
  const float L12 = fmaf(-4.f * kPi * kPi * F, a12, tot.L12);
  const float L22 = fmaf(-2.f * kPi * kPi * F, a22, tot.L22);
  // B = M C0 M^T  ->  dL/dC0 = M^T (dL/dB) M with symmetric dL/dB
  const float m00 = p.cdinv[0], m01 = p.cdinv[1], m10 = p.cdinv[2], m11 = p.cdinv[3];
  const float g11 = L11, g12 = 0.5f * L12, g22 = L22;
  // T = (dL/dB) M
  const float t00 = g11 * m00 + g12 * m10, t01 = g11 * m01 + g12 * m11;
  const float t10 = g12 * m00 + g22 * m10, t11 = g12 * m01 + g22 * m11;
  const float c11g = m00 * t00 + m10 * t10;
  const float c12g = 2.f * (m00 * t01 + m10 * t11);
  const float c22g = m01 * t01 + m11 * t11;
  // C0 = s [[1 + e^2 - 2 e1, 2 e2], [2 e2, 1 + e^2 + 2 e1]], s = r_e^2 / (1 + e)^2
  const float re = p.r_e[gidx], e1 = p.e1[gidx], e2 = p.e2[gidx];
  const float esq = e1 * e1 + e2 * e2, e = sqrtf(esq);
  const float r1e = __builtin_amdgcn_rcpf(1.f + e);
  const float s = re * re * (r1e * r1e);
  const float c11 = s * (1.f + esq - 2.f * e1), c12 = 2.f * s * e2, c22 = s * (1.f + esq + 2.f * e1);
  const float dlogre = 2.f * (c11g * c11 + c12g * c12 + c22g * c22);
  float de1 = 0.f, de2 = 0.f;
  if (e > 0.f) {
    // e1 / e and e2 / e stay correctly rounded divisions: e may be as small
    // as the square root of a denormal
    const float ds1 = -2.f * s * r1e * (e1 / e), ds2 = -2.f * s * r1e * (e2 / e);
    const float a11e = 1.f + esq - 2.f * e1, a22e = 1.f + esq + 2.f * e1;
    de1 = c11g * (ds1 * a11e + s * (2.f * e1 - 2.f)) + c12g * (ds1 * 2.f * e2) +
          c22g * (ds1 * a22e + s * (2.f * e1 + 2.f));
    de2 = c11g * (ds2 * a11e + s * 2.f * e2) + c12g * (ds2 * 2.f * e2 + 2.f * s) +
          c22g * (ds2 * a22e + s * 2.f * e2);
  }
  float* gpo = grad_params + gidx * 6;
  gpo[0] = dxs;
  gpo[1] = dys;
  gpo[2] = tot.dF;
  gpo[3] = dlogre;
  gpo[4] = de1;
  gpo[5] = de2;
}

}  // namespace gfc
