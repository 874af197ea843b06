// Host-side check of the library's fp64 sincos (trig.h) against glibc:
// prints the largest error in ulps of the glibc value over seeded arguments.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "launch.h"
#include "trig.h"

static double ulp_of(double v) {
  double a = fabs(v);
  if (a < 0x1p-1022) return 0x1p-1074;
  return nextafter(a, INFINITY) - a;
}

int main(int argc, char** argv) {
  // "tier dt A B C": the shift tier the host selects for a step
  if (argc == 6 && argv[1][0] == 't') {
    printf("%d\n", soax::shift_tier(atof(argv[2]), atof(argv[3]), atof(argv[4]), atof(argv[5])));
    return 0;
  }
  const double lo = argc > 1 ? atof(argv[1]) : -1.0;
  const double hi = argc > 2 ? atof(argv[2]) : 8.0;
  const long n = argc > 3 ? atol(argv[3]) : 1000000;
  // shifts of the shifted evaluation: |d| < shift_max (default 1/64, the
  // bound of the unchecked form); larger values reach the checked form's
  // longer series (to 1/8) and its full reduction
  const double shift_max = argc > 4 ? atof(argv[4]) : 1.0 / 64;
  uint64_t st = 0x9E3779B97F4A7C15ull;
  double worst_s = 0, worst_c = 0, at_s = 0, at_c = 0;
  for (long i = 0; i < n + 16; ++i) {
    double x;
    if (i < 16) {  // quadrant boundaries and special points
      const double pts[16] = {0.0, -0.0, 1e-300, 1e-8, M_PI / 4, M_PI / 2, M_PI, 3 * M_PI / 2,
                              2 * M_PI, 6.283185307179586, -M_PI / 2, 5e-324, 1.0, -1.0,
                              3.141592653589793, 7.0};
      x = pts[i];
    } else {
      st += 0x9E3779B97F4A7C15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      x = lo + (hi - lo) * ((z >> 11) * 0x1p-53);
    }
    double s, c;
    soax::trig::sincos_fast(x, &s, &c);
    const double es = fabs(s - sin(x)) / ulp_of(sin(x));
    const double ec = fabs(c - cos(x)) / ulp_of(cos(x));
    if (es > worst_s) { worst_s = es; at_s = x; }
    if (ec > worst_c) { worst_c = ec; at_c = x; }
  }
  // shifted evaluation: sin/cos(x + d) from sin/cos(x), reference in long double;
  // the error is absolute, in units of ulp(1) = 2^-52
  double worst_ss = 0, worst_sc = 0;
  long tier_mismatch = 0;
  double worst_small = 0;
  for (long i = 0; i < n; ++i) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double x = lo + (hi - lo) * ((z >> 11) * 0x1p-53);
    // shifts up to shift_max (a few much smaller)
    const double d = ((z & 0x7ff) ? 2 * shift_max : 0x1p-10) * (((z >> 11) & 0xfffff) * 0x1p-20 - 0.5);
    double s, c, s2, c2;
    soax::trig::sincos_fast(x, &s, &c);
    soax::trig::sincos_shift(x, s, c, d, &s2, &c2);
    // inside its bound the mid tier gives exactly the any-tier results
    double s3, c3;
    if (fabs(d) <= soax::trig::kShiftLong) {
      soax::trig::sincos_shift<soax::trig::kTierMid>(x, s, c, d, &s3, &c3);
      if (s3 != s2 || c3 != c2) ++tier_mismatch;
    }
    const long double xl = (long double)x + (long double)d;
    const double rs = (double)sinl(xl), rc = (double)cosl(xl);
    // angle addition bounds the absolute error: measure it in ulps of 1
    const double es = fabs(s2 - rs) / 0x1p-52, ec = fabs(c2 - rc) / 0x1p-52;
    if (es > worst_ss) worst_ss = es;
    if (ec > worst_sc) worst_sc = ec;
    // the small tier's short series, inside its bound
    if (fabs(d) <= soax::trig::kShiftMax) {
      soax::trig::sincos_shift<soax::trig::kTierSmall>(x, s, c, d, &s3, &c3);
      const double e3 = fabs(s3 - rs) / 0x1p-52, f3 = fabs(c3 - rc) / 0x1p-52;
      if (e3 > worst_small) worst_small = e3;
      if (f3 > worst_small) worst_small = f3;
    }
  }
  printf("%.3f %.17g %.3f %.17g %.3f %.3f %ld %.3f\n", worst_s, at_s, worst_c, at_c, worst_ss,
         worst_sc, tier_mismatch, worst_small);
  return 0;
}
