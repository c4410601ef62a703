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

// Radix of the decimation-in-frequency stage working on blocks of length L:
// radix 2 when log2(L) is odd (only the first stage), radix 4 otherwise.
constexpr int dif_radix(int L) { return (ilog2(L) & 1) ? 2 : 4; }

// Position of output k after the DIF stages of a length-L transform.
constexpr int dif_pos(int L, int k) {
  return L == 1 ? 0 : (k % dif_radix(L)) * (L / dif_radix(L)) + dif_pos(L / dif_radix(L), k / dif_radix(L));
}

template <int N, int SIGN, int L>
GFC_HD void dif_stage(float2 (&a)[N]) {
  if constexpr (L >= 2) {
    constexpr int R = dif_radix(L);
    static_for<0, N / L>([&](auto sb) {
      static_for<0, L / R>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        constexpr int base = decltype(sb)::value * L + j;
        if constexpr (R == 2) {
          constexpr int H = L / 2;
          const float2 x0 = a[base], x1 = a[base + H];
          a[base] = cadd(x0, x1);
          a[base + H] = twiddle<SIGN, L, j>(csub(x0, x1));
        } else {
          constexpr int Q = L / 4;
          const float2 x0 = a[base], x1 = a[base + Q], x2 = a[base + 2 * Q], x3 = a[base + 3 * Q];
          const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
          const float2 t2 = cadd(x1, x3), t3 = rot90<SIGN>(csub(x1, x3));
          a[base] = cadd(t0, t2);
          a[base + Q] = twiddle<SIGN, L, j>(cadd(t1, t3));
          a[base + 2 * Q] = twiddle<SIGN, L, 2 * j>(csub(t0, t2));
          a[base + 3 * Q] = twiddle<SIGN, L, 3 * j>(csub(t1, t3));
        }
      });
    });
    dif_stage<N, SIGN, L / R>(a);
  }
}

// In-place unnormalised DFT of length N (power of two, 1..256):
//   a[k] <- sum_n a[n] exp(SIGN * 2 pi i k n / N),  natural order in and out.
template <int N, int SIGN>
GFC_HD void fft(float2 (&a)[N]) {
  dif_stage<N, SIGN, N>(a);
  float2 t[N];
  static_for<0, N>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    t[k] = a[dif_pos(N, k)];
  });
  static_for<0, N>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    a[k] = t[k];
  });
}

// Runtime twiddle exp(SIGN * 2 pi i k / L) for a lane-dependent k (table lookup).
template <int SIGN, int L>
__device__ __forceinline__ float2 twiddle_rt(int k) {
  const int t = (k & (L - 1)) * (GFC_TW_N / L);
  const float s = kTwSinRt[t];
  return make_float2(kTwCosRt[t], SIGN > 0 ? s : -s);
}

}  // namespace gfc
