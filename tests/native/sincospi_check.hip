// Host-side check of the kernels' sincospi polynomial (gfc::sincospi_poly):
// prints the largest absolute errors against double-precision sin/cos(pi r)
// over a dense sweep of the arguments the kernels use (|r| <= 512) and a
// random sample, and counts violations of the exact values and symmetries.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "gfc_device.hpp"

static double ref_reduced(double r) { return r - 2.0 * std::floor(r / 2.0); }

int main() {
  double es = 0, ec = 0;
  long bad_exact = 0, bad_sym = 0;
  auto check = [&](float r) {
    float s, c;
    gfc::sincospi_poly(r, &s, &c);
    const double rr = ref_reduced((double)r);
    es = std::fmax(es, std::fabs(s - std::sin(M_PI * rr)));
    ec = std::fmax(ec, std::fabs(c - std::cos(M_PI * rr)));
    float s2, c2;
    gfc::sincospi_poly(-r, &s2, &c2);
    if (s2 != -s || c2 != c) ++bad_sym;
  };
  for (long i = 0; i <= 8000000; ++i) check((float)(i * (512.0 / 8000000.0)));
  uint32_t x = 12345u;
  for (long i = 0; i < 4000000; ++i) {
    x = x * 1664525u + 1013904223u;
    check(((float)(x >> 8) * (1.0f / 16777216.0f) - 0.5f) * (float)(2 * ((i % 9) + 1)));
  }
  for (int k = -512; k <= 512; ++k) {  // sin(pi k) = 0, cos(pi k) = (-1)^k, and the half turns
    float s, c;
    gfc::sincospi_poly((float)k, &s, &c);
    if (s != 0.f || c != ((k & 1) ? -1.f : 1.f)) ++bad_exact;
    gfc::sincospi_poly((float)k + 0.5f, &s, &c);
    if (c != 0.f || s != ((k & 1) ? -1.f : 1.f)) ++bad_exact;
  }
  std::printf("%.6e %.6e %ld %ld\n", es, ec, bad_exact, bad_sym);
  return 0;
}
