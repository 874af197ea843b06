// Device-versus-host check of the library's fp64 sine/cosine (trig.h).
//
// The GPU evaluates the sine and cosine series as one inline-asm block of
// v_fma_f64 instructions; the host build of the same header evaluates them
// with fma() calls.  Both are chains of correctly rounded fused multiply-adds
// on the same operands, so the two must agree bit for bit.  This helper runs
// sincos_fast and sincos_shift in each of its tiers (|d| <= 1/64; |f| below
// 1/8; any e) on seeded arguments on the GPU and on the host and counts the
// results whose bits differ.  Test infrastructure only: it is
// compiled by the test build and loaded by the GPU tests through ctypes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "trig.h"

namespace {

constexpr int kOut = 8;  // sin, cos of x; of x + d (small tier); of x + e (any); of x + f (mid)

__global__ void trig_kernel(const double* x, const double* d, const double* e, const double* f,
                            double* out, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c, r[kOut];
  soax::trig::sincos_fast(x[i], &s, &c);
  r[0] = s;
  r[1] = c;
  soax::trig::sincos_shift<soax::trig::kTierSmall>(x[i], s, c, d[i], &r[2], &r[3]);
  soax::trig::sincos_shift<soax::trig::kTierAny>(x[i], s, c, e[i], &r[4], &r[5]);
  soax::trig::sincos_shift<soax::trig::kTierMid>(x[i], s, c, f[i], &r[6], &r[7]);
  for (int k = 0; k < kOut; ++k) out[i * kOut + k] = r[k];
}

// SplitMix64 (Steele, Lea and Flood, 2014): a uniform double in [0, 1).
double uniform(uint64_t* st) {
  *st += 0x9E3779B97F4A7C15ull;
  uint64_t z = *st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return static_cast<double>(z >> 11) * 0x1p-53;
}

}  // namespace

// n arguments x uniform in [lo, hi) (the first 12 replaced by quadrant
// boundaries and special points inside the range), small-tier shifts d
// uniform in [-1/64, 1/64], any-tier shifts e uniform in [-emax, emax],
// mid-tier shifts f uniform in [-m, m] with m = min(emax, 1/8).  mismatch[k]
// counts results of kind k (see kOut) whose bits differ between the GPU and
// the host; first_x[k] is the first such argument.  Returns a hipError_t code.
extern "C" int trig_device_check(int64_t n, double lo, double hi, double emax, uint64_t seed,
                                 int64_t* mismatch, double* first_x) {
  if (n <= 0) return hipErrorInvalidValue;
  std::vector<double> x(n), d(n), e(n), f(n), got(n * kOut);
  const double fmax = emax < soax::trig::kShiftLong ? emax : soax::trig::kShiftLong;
  uint64_t st = seed;
  const double special[12] = {0.0, -0.0, 1e-300, 0.7853981633974483, 1.5707963267948966,
                              3.141592653589793, 4.71238898038469, 6.283185307179586,
                              -1.5707963267948966, 5e-324, 1.0, -1.0};
  for (int64_t i = 0; i < n; ++i) {
    x[i] = lo + (hi - lo) * uniform(&st);
    if (i < 12 && special[i] >= lo && special[i] < hi) x[i] = special[i];
    d[i] = (2.0 * uniform(&st) - 1.0) * soax::trig::kShiftMax;
    e[i] = (2.0 * uniform(&st) - 1.0) * emax;
    f[i] = (2.0 * uniform(&st) - 1.0) * fmax;
  }
  double *dx = nullptr, *dd = nullptr, *de = nullptr, *df = nullptr, *dout = nullptr;
  hipError_t err = hipSuccess;
  const size_t bytes = sizeof(double) * n;
  if ((err = hipMalloc(&dx, bytes)) != hipSuccess) goto done;
  if ((err = hipMalloc(&dd, bytes)) != hipSuccess) goto done;
  if ((err = hipMalloc(&de, bytes)) != hipSuccess) goto done;
  if ((err = hipMalloc(&df, bytes)) != hipSuccess) goto done;
  if ((err = hipMalloc(&dout, bytes * kOut)) != hipSuccess) goto done;
  if ((err = hipMemcpy(dx, x.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) goto done;
  if ((err = hipMemcpy(dd, d.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) goto done;
  if ((err = hipMemcpy(de, e.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) goto done;
  if ((err = hipMemcpy(df, f.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) goto done;
  hipLaunchKernelGGL(trig_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, 0,
                     dx, dd, de, df, dout, n);
  if ((err = hipGetLastError()) != hipSuccess) goto done;
  if ((err = hipMemcpy(got.data(), dout, bytes * kOut, hipMemcpyDeviceToHost)) != hipSuccess)
    goto done;
  for (int k = 0; k < kOut; ++k) {
    mismatch[k] = 0;
    first_x[k] = 0.0;
  }
  for (int64_t i = 0; i < n; ++i) {
    double s, c, r[kOut];
    soax::trig::sincos_fast(x[i], &s, &c);
    r[0] = s;
    r[1] = c;
    soax::trig::sincos_shift<soax::trig::kTierSmall>(x[i], s, c, d[i], &r[2], &r[3]);
    soax::trig::sincos_shift<soax::trig::kTierAny>(x[i], s, c, e[i], &r[4], &r[5]);
    soax::trig::sincos_shift<soax::trig::kTierMid>(x[i], s, c, f[i], &r[6], &r[7]);
    for (int k = 0; k < kOut; ++k)
      if (memcmp(&r[k], &got[i * kOut + k], sizeof(double)) != 0 && mismatch[k]++ == 0)
        first_x[k] = x[i];
  }
done:
  hipFree(dx);
  hipFree(dd);
  hipFree(de);
  hipFree(df);
  hipFree(dout);
  return static_cast<int>(err);
}
