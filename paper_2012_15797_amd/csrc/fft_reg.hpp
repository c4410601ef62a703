// In-register radix-4/2 FFTs for one lane, fully unrolled at compile time.
//
// Every index is a compile-time constant, so the arrays live in VGPRs and
// every twiddle factor is an immediate operand; multiplications by 1, -1 and
// +-i are resolved at compile time into moves and sign flips.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "twiddles.inc"

namespace gfc {

#define GFC_HD __host__ __device__ __forceinline__

// ------------------------------------------------------------ compile-time loops
template <int B, int E, typename F, int... I>
GFC_HD void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, B + I>{}), ...);
}
template <int B, int E, typename F>
GFC_HD void static_for(F&& f) {
  if constexpr (E > B) static_for_impl<B, E>(static_cast<F&&>(f), std::make_integer_sequence<int, E - B>{});
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// ------------------------------------------------------------ complex helpers
GFC_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
GFC_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
GFC_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
GFC_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
GFC_HD float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
GFC_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
// a b + c in four FMAs
GFC_HD float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
// multiply by SIGN * i
template <int SIGN>
GFC_HD float2 rot90(float2 v) {
  if constexpr (SIGN > 0) return make_float2(-v.y, v.x);
  else return make_float2(v.y, -v.x);
}

// v * exp(SIGN * 2 pi i * IDX / L), L a power of two dividing 256.
template <int SIGN, int L, int IDX>
GFC_HD float2 twiddle(float2 v) {
  constexpr int k = ((IDX % L) + L) % L;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (4 * k == L) {
    return rot90<SIGN>(v);
  } else if constexpr (2 * k == L) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * k == 3 * L) {
    return rot90<-SIGN>(v);
  } else {
    static_assert(GFC_TW_N % L == 0, "twiddle table too small");
    constexpr int t = k * (GFC_TW_N / L);
    constexpr float c = kTwCos[t];
    constexpr float s = SIGN > 0 ? kTwSin[t] : -kTwSin[t];
    return make_float2(fmaf(v.x, c, -(v.y * s)), fmaf(v.x, s, v.y * c));
  }
}

// A twiddle w = exp(SIGN 2 pi i K / L) as a real scale r times a factor
// applied by unit(v), so that w v = r unit(v).  For 1, -1 and +-i, r = 1 and
// unit is the exact product.  Otherwise w = r (1 + i q) when |cos| >= |sin|,
// else r (q + i), with |q| <= 1 (the tangent or cotangent), and unit takes
// two FMAs: a product w v that feeds an add then folds into FMAs.
template <int SIGN, int L, int K>
struct TwFactor {
  static constexpr int k = ((K % L) + L) % L;
  static constexpr bool trivial = (4 * k) % L == 0;
  static constexpr int t = trivial ? 0 : k * (GFC_TW_N / L);
  static constexpr float c = kTwCos[t];
  static constexpr float s = SIGN > 0 ? kTwSin[t] : -kTwSin[t];
  static constexpr bool by_cos = (c >= 0.f ? c : -c) >= (s >= 0.f ? s : -s);
  static constexpr float r = trivial ? 1.f : (by_cos ? c : s);
  static constexpr float q = SIGN > 0 ? kTwRatio[t] : -kTwRatio[t];
  static GFC_HD float2 unit(float2 v) {
    if constexpr (trivial) return twiddle<SIGN, L, K>(v);
    else if constexpr (by_cos) return make_float2(fmaf(-q, v.y, v.x), fmaf(q, v.x, v.y));
    else return make_float2(fmaf(q, v.x, -v.y), fmaf(q, v.y, v.x));
  }
};

// Radix-2 butterfly (a, b) <- (a + w b, a - w b), w = exp(SIGN 2 pi i K / L):
// four adds when w is 1, -1 or +-i, otherwise six FMAs (w b = r u with
// u = unit(b), then a +- r u), against four adds and a complex product.
template <int SIGN, int L, int K>
GFC_HD void bfly2(float2& a, float2& b) {
  constexpr int k = ((K % L) + L) % L;
  const float2 p = a;
  if constexpr (k == 0) {
    a = cadd(p, b);
    b = csub(p, b);
  } else if constexpr (2 * k == L) {
    a = csub(p, b);
    b = cadd(p, b);
  } else if constexpr (4 * k == L || 4 * k == 3 * L) {
    const float2 wb = (4 * k == L) ? rot90<SIGN>(b) : rot90<-SIGN>(b);
    a = cadd(p, wb);
    b = csub(p, wb);
  } else {
    static_assert(GFC_TW_N % L == 0, "twiddle table too small");
    using T = TwFactor<SIGN, L, k>;
    static_assert(!T::trivial, "trivial twiddles take the branches above");
    const float2 u = T::unit(b);
    a = make_float2(fmaf(T::r, u.x, p.x), fmaf(T::r, u.y, p.y));
    b = make_float2(fmaf(-T::r, u.x, p.x), fmaf(-T::r, u.y, p.y));
  }
}

// Pair step of a complex-to-real inverse transform run as a half-length
// complex FFT: with s = a + b, t = w (a - b), w = exp(SIGN 2 pi i K / L),
// lo = s + i t and hi = conj(s) + i conj(t).  t = r u (TwFactor), so each
// output component is one FMA.
template <int SIGN, int L, int K>
GFC_HD void c2r_pair(float2 a, float2 b, float2& lo, float2& hi) {
  using T = TwFactor<SIGN, L, K>;
  const float2 sum = cadd(a, b);
  const float2 u = T::unit(csub(a, b));
  lo = make_float2(fmaf(-T::r, u.y, sum.x), fmaf(T::r, u.x, sum.y));
  hi = make_float2(fmaf(T::r, u.y, sum.x), fmaf(T::r, u.x, -sum.y));
}

// Radix of the stage combining sub-transforms into blocks of length L: 2 for
// the first stage of an odd power of two (L = 2), 4 otherwise, so the
// largest blocks, where most twiddles are non-trivial, are radix 4.
constexpr int stage_radix(int L) { return L == 2 ? 2 : 4; }

// Register holding input n of a length-L transform before the stages run
// (mixed-radix digit reversal): block p of length L/R holds the
// sub-sequence n = p (mod R), recursively.
constexpr int in_pos(int L, int n) {
  return L == 1 ? 0 : (n % stage_radix(L)) * (L / stage_radix(L)) + in_pos(L / stage_radix(L), n / stage_radix(L));
}

// Radix-4 butterfly j of a block of length L on element j of the four
// sub-transforms X0..X3, w = exp(SIGN 2 pi i / L), w^(L/4) = SIGN i:
//   t0, t1 = X0 +- w^2j X2;   b1 +- b3 = w^j X1 +- w^3j X3;
//   y0, y2 = t0 +- (b1 + b3); y1, y3 = t1 +- SIGN i (b1 - b3).
// With w^j = r1 unit1, w^3j = r3 unit3 (TwFactor), b1 +- b3 = r1 (u1 +- (r3/r1) u3),
// so every product folds into an FMA: 22 instructions when all three
// twiddles are non-trivial, against 24 for four radix-2 butterflies.
template <int SIGN, int L, int J>
GFC_HD void bfly4(float2& x0, float2& x1, float2& x2, float2& x3) {
  using T1 = TwFactor<SIGN, L, J>;
  using T3 = TwFactor<SIGN, L, 3 * J>;
  if constexpr (T1::trivial || T3::trivial) {
    // j = 0 (all trivial): the plain radix-4 butterfly
    bfly2<SIGN, L, 2 * J>(x0, x2);
    bfly2<SIGN, L, 2 * J>(x1, x3);
    bfly2<SIGN, L, J>(x0, x1);
    bfly2<SIGN, L, J + L / 4>(x2, x3);
    const float2 t = x1;
    x1 = x2;
    x2 = t;
  } else {
    bfly2<SIGN, L, 2 * J>(x0, x2);  // x0 = t0, x2 = t1
    constexpr float rho = T3::r / T1::r;
    const float2 u1 = T1::unit(x1), u3 = T3::unit(x3);
    const float2 sp = make_float2(fmaf(rho, u3.x, u1.x), fmaf(rho, u3.y, u1.y));
    const float2 dp = make_float2(fmaf(-rho, u3.x, u1.x), fmaf(-rho, u3.y, u1.y));
    constexpr float r = T1::r;
    constexpr float ri = SIGN > 0 ? T1::r : -T1::r;  // SIGN i r1 dp = (-ri dp.y, ri dp.x)
    const float2 t0 = x0, t1 = x2;
    x0 = make_float2(fmaf(r, sp.x, t0.x), fmaf(r, sp.y, t0.y));
    x2 = make_float2(fmaf(-r, sp.x, t0.x), fmaf(-r, sp.y, t0.y));
    x1 = make_float2(fmaf(-ri, dp.y, t1.x), fmaf(ri, dp.x, t1.y));
    x3 = make_float2(fmaf(ri, dp.y, t1.x), fmaf(-ri, dp.x, t1.y));
  }
}

// Decimation-in-time stages up to block length L: the blocks of length L/R
// hold the R sub-transforms, and butterfly j of a block forms outputs
// j + (L/R) q from element j of each.  The twiddles meet the inputs of the
// butterflies, where they fold into FMAs (bfly2, bfly4).
template <int N, int SIGN, int L>
GFC_HD void dit_stages(float2 (&a)[N]) {
  if constexpr (L >= 2) {
    constexpr int R = stage_radix(L);
    dit_stages<N, SIGN, L / R>(a);
    static_for<0, N / L>([&](auto sb) {
      static_for<0, L / R>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int base = decltype(sb)::value * L + j;
        if constexpr (R == 2) {
          bfly2<SIGN, L, j>(a[base], a[base + L / 2]);
        } else {
          constexpr int Q = L / 4;
          bfly4<SIGN, L, j>(a[base], a[base + Q], a[base + 2 * Q], a[base + 3 * Q]);
        }
      });
    });
  }
}

// In-place unnormalised DFT of length N (power of two, 1..256):
//   a[k] <- sum_n a[n] exp(SIGN 2 pi i k n / N),  natural order in and out.
// The input permutation is a renaming of registers and costs nothing.
template <int N, int SIGN>
GFC_HD void fft(float2 (&a)[N]) {
  float2 t[N];
  static_for<0, N>([&](auto nn) {
    constexpr int n = decltype(nn)::value;
    t[in_pos(N, n)] = a[n];
  });
  static_for<0, N>([&](auto nn) {
    constexpr int n = decltype(nn)::value;
    a[n] = t[n];
  });
  dit_stages<N, SIGN, N>(a);
}

// Runtime twiddle exp(SIGN * 2 pi i k / L) for a lane-dependent k (table lookup).
template <int SIGN, int L>
__device__ __forceinline__ float2 twiddle_rt(int k) {
  const int t = (k & (L - 1)) * (GFC_TW_N / L);
  const float s = kTwSinRt[t];
  return make_float2(kTwCosRt[t], SIGN > 0 ? s : -s);
}

}  // namespace gfc
