// trig.h -- fp64 sine and cosine for the hot path.
//
// sincos_fast(x): both functions of one argument.  Positions on the hot path
// stay within a few box edges of the origin, so the full-range reduction of
// the device math library (Payne-Hanek) is replaced for |x| <= 2^19 by the
// Cody-Waite method (W. J. Cody and W. Waite, "Software Manual for the
// Elementary Functions", 1980):
//   k = nearest integer to x * 2/pi,  r = x - k*pi/2  with pi/2 split into
//   three doubles (the first two with 33 significant bits, so k*part is exact
//   for |k| < 2^20; constants derived by gen_trig_constants.py),
// followed by the Taylor series of sin and cos on |r| <= pi/4, truncated
// after r^15 and r^16 (the first omitted terms, r^17/17! and r^18/18!, are at
// most 6.6e-17 relative for sin and 2.9e-18 for cos), evaluated by Horner's
// rule.  The quadrant k mod 4 picks and signs the
// results.  Arguments outside that range, infinities and NaNs go to the
// device library's sincos.
//
// sincos_shift(x, sin x, cos x, d): both functions of x + d for a small shift
// |d| <= 1/64, by the angle-addition formulas with sin d and cos d - 1 from
// their Taylor series (truncated after d^5 and d^6; omitted terms below
// 5e-17 absolute).  A time step moves a particle by dt*u, far less than 1/64
// for the step sizes of interest, so the midpoint and end-point values of a
// step come from the start-point values without a second reduction.  Where
// shifts may exceed 1/64 the longer series (truncated after d^9 and d^10)
// take every shift up to 1/8, and larger shifts fall back to
// sincos_fast(x + d) (see the tiers below).  The shift uses the exact sum
// x + d, which differs from the rounded sum by at most half an ulp of x.
//
// Measured on the host against glibc over seeded arguments: within 2 ulp for
// |x| up to 2^19 (the 2-ulp cases at large |x|, where the reduction's error
// grows with k), and the shifted forms within one ulp of 1 in absolute error.
// The GPU's results equal the host build's bit for bit (both are chains of
// correctly rounded fmas).
#pragma once

#include <hip/hip_runtime.h>

namespace soax {
namespace trig {

constexpr double kPio2Hi = 0x1.921fb54400000p+0;
constexpr double kPio2Mid = 0x1.0b4611a600000p-34;
constexpr double kPio2Lo = 0x1.3198a2e037073p-69;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kFastMax = 0x1p19;
constexpr double kShiftMax = 1.0 / 64;

// 1/n! rounded once: n! is exact in a double for n <= 18.
constexpr double inv_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}

// sin r = r + r^3 (S1 + w (S2 + ... + w^5 S7)),  w = r^2
constexpr double S1 = -inv_fact(3), S2 = inv_fact(5), S3 = -inv_fact(7), S4 = inv_fact(9),
                 S5 = -inv_fact(11), S6 = inv_fact(13), S7 = -inv_fact(15);
// cos r = 1 - w/2 + w^2 (C1 + w (C2 + ... + w^5 C7))
constexpr double C1 = inv_fact(4), C2 = -inv_fact(6), C3 = inv_fact(8), C4 = -inv_fact(10),
                 C5 = inv_fact(12), C6 = -inv_fact(14), C7 = inv_fact(16);

struct SinCos {
  double s, c;
};

// The two series' Horner chains in w: ps = S1 + w (S2 + ... + w S7) and
// pc = C1 + w (C2 + ... + w C7), each step one fma.  On the GPU both chains
// run interleaved in one block of three-operand fmas (the top step's added
// constant from a vector register, every other constant a scalar-register
// operand): the compiler cannot see into separate asm statements and pads
// each dependent pair of them with a wait, which one block does not need.
__host__ __device__ __forceinline__ void sin_cos_series(double w, double& ps, double& pc) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm("v_fma_f64 %0, %2, %3, %4\n\t"
      "v_fma_f64 %1, %2, %5, %6\n\t"
      "v_fma_f64 %0, %2, %0, %7\n\t"
      "v_fma_f64 %1, %2, %1, %8\n\t"
      "v_fma_f64 %0, %2, %0, %9\n\t"
      "v_fma_f64 %1, %2, %1, %10\n\t"
      "v_fma_f64 %0, %2, %0, %11\n\t"
      "v_fma_f64 %1, %2, %1, %12\n\t"
      "v_fma_f64 %0, %2, %0, %13\n\t"
      "v_fma_f64 %1, %2, %1, %14\n\t"
      "v_fma_f64 %0, %2, %0, %15\n\t"
      "v_fma_f64 %1, %2, %1, %16"
      : "=&v"(ps), "=&v"(pc)
      : "v"(w), "s"(S7), "v"(S6), "s"(C7), "v"(C6), "s"(S5), "s"(C5), "s"(S4), "s"(C4),
        "s"(S3), "s"(C3), "s"(S2), "s"(C2), "s"(S1), "s"(C1));
#else
  ps = fma(w, fma(w, fma(w, fma(w, fma(w, fma(w, S7, S6), S5), S4), S3), S2), S1);
  pc = fma(w, fma(w, fma(w, fma(w, fma(w, fma(w, C7, C6), C5), C4), C3), C2), C1);
#endif
}

// Out-of-range arguments: kept out of line so the fast path stays small.  The
// pair is returned by value so that the caller's results never have to live
// in memory.
inline __host__ __device__ __attribute__((noinline)) SinCos sincos_wide(double x) {
  SinCos r;
  sincos(x, &r.s, &r.c);
  return r;
}

__host__ __device__ __forceinline__ void sincos_fast(double x, double* s, double* c) {
  if (!(fabs(x) <= kFastMax)) {
    const SinCos r = sincos_wide(x);
    *s = r.s;
    *c = r.c;
    return;
  }
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, kPio2Hi, x);  // exact
  r = fma(-k, kPio2Mid, r);
  r = fma(-k, kPio2Lo, r);
  const double w = r * r;
  double ps, pc;
  sin_cos_series(w, ps, pc);
  const double sr = fma(r * w, ps, r);
  const double cr = fma(w, fma(w, pc, -0.5), 1.0);
  // x = k pi/2 + r:  sin x = (sr, cr, -sr, -cr)[k mod 4], cos x = (cr, -sr, -cr, sr)[k mod 4]
  const uint32_t q = static_cast<uint32_t>(static_cast<int>(k));
  // bit 0 of q (swap sr and cr) and bit 1 (the sine's sign) moved to bit 31;
  // the cosine's sign is bit 1 of q + 1, i.e. bit 1 xor bit 0
  const uint32_t odd = q << 31;
  const uint32_t hs = (q << 30) & 0x80000000u;
  const uint32_t hc = hs ^ odd;
  const double a = odd ? cr : sr;
  const double b = odd ? sr : cr;
  *s = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, a) ^ (static_cast<uint64_t>(hs) << 32));
  *c = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, b) ^ (static_cast<uint64_t>(hc) << 32));
}

// sin d = d + d^3 (T1 + w T2)
constexpr double T1 = -inv_fact(3), T2 = inv_fact(5);
// cos d - 1 = w (-1/2 + w (U1 + w U2))
constexpr double U1 = inv_fact(4), U2 = -inv_fact(6);
// the longer series, for |d| <= 1/8:
// sin d = d + d^3 (T1 + w (T2 + w (T3 + w T4))), omitted terms below 3e-18;
// cos d - 1 = w (-1/2 + w (U1 + w (U2 + w (U3 + w U4)))), below 3e-20
constexpr double kShiftLong = 1.0 / 8;
constexpr double T3 = -inv_fact(7), T4 = inv_fact(9);
constexpr double U3 = inv_fact(8), U4 = -inv_fact(10);

// What the caller guarantees about the shift, by tier.  kTierSmall:
// |d| <= kShiftMax; the short series.  kTierMid: |d| <= kShiftLong; the
// longer series for every shift (no branch, so the lanes of a wave never
// split between two series).  kTierAny: any d; the longer series up to
// kShiftLong and a full reduction of x + d beyond it.  Where its guarantee
// holds, kTierMid gives exactly the results of kTierAny.
constexpr int kTierSmall = 0;
constexpr int kTierMid = 1;
constexpr int kTierAny = 2;

template <int TIER = kTierAny>
__host__ __device__ __forceinline__ void sincos_shift(double x, double sx, double cx, double d,
                                                      double* s, double* c) {
  double sd, cm1;
  const double w = d * d;
  if (TIER == kTierSmall) {
    sd = fma(d * w, fma(w, T2, T1), d);
    cm1 = w * fma(w, fma(w, U2, U1), -0.5);
  } else {
    if (TIER == kTierAny && !(fabs(d) <= kShiftLong)) {
      sincos_fast(x + d, s, c);
      return;
    }
    sd = fma(d * w, fma(w, fma(w, fma(w, T4, T3), T2), T1), d);
    cm1 = w * fma(w, fma(w, fma(w, fma(w, U4, U3), U2), U1), -0.5);
  }
  // sin(x+d) = sin x + (sin x (cos d - 1) + cos x sin d), likewise for cos
  *s = fma(cx, sd, fma(sx, cm1, sx));
  *c = fma(-sx, sd, fma(cx, cm1, cx));
}

}  // namespace trig
}  // namespace soax
