// Host-side check of the kernels' in-register FFTs (gfc::fft<N, SIGN>, the
// decimation-in-time stages with FMA butterflies): for every power-of-two
// length 1..256 and both signs, the largest error against a
// double-precision direct DFT of the same float inputs, relative to the
// largest output magnitude, over several seeded random vectors, plus two
// exact cases (a unit impulse transforms to all ones, a constant to N at
// bin 0).  Prints one line per (N, SIGN): N SIGN rel_err exact_failures.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "fft_reg.hpp"

static uint32_t g_state = 2024u;
static float urand() {  // uniform in [-1, 1)
  g_state = g_state * 1664525u + 1013904223u;
  return (float)(g_state >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

template <int N, int SIGN>
static void check() {
  double worst = 0.0;
  for (int trial = 0; trial < 20; ++trial) {
    float2 a[N];
    double xr[N], xi[N];
    for (int n = 0; n < N; ++n) {
      a[n] = make_float2(urand(), urand());
      xr[n] = a[n].x;
      xi[n] = a[n].y;
    }
    gfc::fft<N, SIGN>(a);
    double peak = 0.0, err = 0.0;
    for (int k = 0; k < N; ++k) {
      double sr = 0.0, si = 0.0;
      for (int n = 0; n < N; ++n) {
        const double ang = SIGN * 2.0 * M_PI * (double)((long)k * n % N) / N;
        sr += xr[n] * std::cos(ang) - xi[n] * std::sin(ang);
        si += xr[n] * std::sin(ang) + xi[n] * std::cos(ang);
      }
      peak = std::fmax(peak, std::hypot(sr, si));
      err = std::fmax(err, std::hypot(a[k].x - sr, a[k].y - si));
    }
    worst = std::fmax(worst, err / peak);
  }
  long bad = 0;
  {
    float2 a[N];
    for (int n = 0; n < N; ++n) a[n] = make_float2(n == 0 ? 1.f : 0.f, 0.f);
    gfc::fft<N, SIGN>(a);
    for (int k = 0; k < N; ++k) bad += (a[k].x != 1.f || a[k].y != 0.f);
    for (int n = 0; n < N; ++n) a[n] = make_float2(1.f, 0.f);
    gfc::fft<N, SIGN>(a);
    for (int k = 0; k < N; ++k) bad += std::fabs(a[k].x - (k == 0 ? (float)N : 0.f)) > 1e-5f * N || std::fabs(a[k].y) > 1e-5f * N;
  }
  std::printf("%d %d %.6e %ld\n", N, SIGN, worst, bad);
}

template <int N>
static void both() {
  check<N, +1>();
  check<N, -1>();
}

int main() {
  both<1>();
  both<2>();
  both<4>();
  both<8>();
  both<16>();
  both<32>();
  both<64>();
  both<128>();
  both<256>();
  return 0;
}
