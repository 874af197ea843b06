// host_adjoint.cpp -- host side of the checkpointed RK2 forward, the
// discrete adjoint and the loss (SoA arrays or positions inside records).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host_internal.h"

using namespace soax;
using namespace soax::host;

extern "C" {

// ------------------------------------------------------------- adjoints

static soax_status check_abc_host(const double* abc) {
  if (!abc) return fail(SOAX_E_ARG, "abc is NULL");
  if (!is_finite(abc[0]) || !is_finite(abc[1]) || !is_finite(abc[2]))
    return fail(SOAX_E_ARG, "field amplitudes must be finite");
  return SOAX_OK;
}

static soax_status check_rows(const void* const* rows, int64_t n, const char* what) {
  if (!rows) return fail(SOAX_E_ARG, "%s is NULL", what);
  if (n > 0)
    for (int d = 0; d < 3; ++d)
      if (!rows[d]) return fail(SOAX_E_ARG, "%s[%d] is NULL", what, d);
  return SOAX_OK;
}

static soax_status check_stride(int64_t stride) {
  if (stride < 1 || stride > 4096) return fail(SOAX_E_ARG, "stride %lld outside 1..4096", static_cast<long long>(stride));
  return SOAX_OK;
}

soax_status soax_rk2_forward_ckpt_strided(const double* const* x0, double* const* xT, int64_t n,
                                          int64_t stride, const double* abc, double dt,
                                          int64_t nsteps, int64_t k, double* tape, void* stream) {
  soax_status st;
  if ((st = check_stride(stride))) return st;
  if ((st = check_rows(reinterpret_cast<const void* const*>(x0), n, "x0")) ||
      (st = check_rows(reinterpret_cast<const void* const*>(xT), n, "xT")) ||
      (st = check_abc_host(abc)))
    return st;
  if (n < 0 || n > kMaxParticles) return fail(n < 0 ? SOAX_E_ARG : SOAX_E_RANGE, "bad n");
  if (nsteps < 0 || k < 1) return fail(SOAX_E_ARG, "need nsteps >= 0 and k >= 1");
  if (!is_finite(dt)) return fail(SOAX_E_ARG, "dt is not finite");
  if (!tape && n > 0 && nsteps > 0) return fail(SOAX_E_ARG, "tape is NULL");
  CkptArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.x0[d] = x0[d];
    a.xT[d] = xT[d];
  }
  a.tape = tape;
  a.stride = stride;
  a.n = n;
  a.nsteps = nsteps;
  a.k = k;
  a.dt = dt;
  a.abc = AbcParams{abc[0], abc[1], abc[2]};
  HIP_TRY(launch_rk2_forward_ckpt(a, as_stream(stream)), "forward launch");
  return SOAX_OK;
}

soax_status soax_rk2_forward_ckpt(const double* const* x0, double* const* xT, int64_t n,
                                  const double* abc, double dt, int64_t nsteps, int64_t k,
                                  double* tape, void* stream) {
  return soax_rk2_forward_ckpt_strided(x0, xT, n, 1, abc, dt, nsteps, k, tape, stream);
}

soax_status soax_adjoint_strided(const double* tape, const double* const* lamT, int64_t n,
                                 int64_t stride, const double* abc, double dt, int64_t nsteps,
                                 int64_t k, double* const* grad_x0, double* grad_abc,
                                 void* stream) {
  soax_status st;
  if ((st = check_stride(stride))) return st;
  if ((st = check_rows(reinterpret_cast<const void* const*>(lamT), n, "lamT")) ||
      (st = check_rows(reinterpret_cast<const void* const*>(grad_x0), n, "grad_x0")) ||
      (st = check_abc_host(abc)))
    return st;
  if (!grad_abc) return fail(SOAX_E_ARG, "grad_abc is NULL");
  if (n < 0 || n > kMaxParticles) return fail(n < 0 ? SOAX_E_ARG : SOAX_E_RANGE, "bad n");
  if (nsteps < 0 || k < 1) return fail(SOAX_E_ARG, "need nsteps >= 0 and k >= 1");
  if (!is_finite(dt)) return fail(SOAX_E_ARG, "dt is not finite");
  if (!tape && n > 0 && nsteps > 0) return fail(SOAX_E_ARG, "tape is NULL");
  hipStream_t s = as_stream(stream);
  const int64_t parts = std::max<int64_t>(adjoint_partials(n), 1);
  void* partial = nullptr;
  hipError_t e = hipMallocAsync(&partial, parts * 3 * sizeof(double), s);
  if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMallocAsync(partials): %s", hipGetErrorString(e));
  AdjointArgs a{};
  a.tape = tape;
  for (int d = 0; d < 3; ++d) {
    a.lam[d] = lamT[d];
    a.gx[d] = grad_x0[d];
  }
  a.partial = static_cast<double*>(partial);
  a.grad_abc = grad_abc;
  a.stride = stride;
  a.n = n;
  a.nsteps = nsteps;
  a.k = k;
  a.dt = dt;
  a.abc = AbcParams{abc[0], abc[1], abc[2]};
  e = launch_adjoint(a, s);
  hipError_t e2 = hipFreeAsync(partial, s);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync(partials)");
  return SOAX_OK;
}

soax_status soax_adjoint(const double* tape, const double* const* lamT, int64_t n,
                         const double* abc, double dt, int64_t nsteps, int64_t k,
                         double* const* grad_x0, double* grad_abc, void* stream) {
  return soax_adjoint_strided(tape, lamT, n, 1, abc, dt, nsteps, k, grad_x0, grad_abc, stream);
}

// ------------------------------------------- allocation-free adjoint

// Device memory of soax_adjoint_noalloc: the adjoint kernel's per-workgroup
// partial sums of dL/d(A,B,C), three doubles per workgroup of 256 particles,
// in a fixed array that every GPU the library runs on holds until the
// process ends.  Host code never passes `scratch` itself to a kernel (on
// the host the name stands for a host-side symbol, not a device address):
// it passes the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocScratchBytes = int64_t(1) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];  // per device, set once

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
static soax_status scratch_ptr(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SOAX_E_STATE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return SOAX_OK;
}

// Particles whose partial sums fit the scratch: one triple per workgroup.
static_assert(SOAX_ADJOINT_NOALLOC_MAX_N ==
                  kNoAllocScratchBytes / (3 * int64_t(sizeof(double))) * kAdjointBlock,
              "the header's limit must match the scratch size");

soax_status soax_adjoint_noalloc(const double* tape, const double* const* lamT, int64_t n,
                                 const double* abc, double dt, int64_t nsteps, int64_t k,
                                 double* const* grad_x0, double* grad_abc, void* stream) {
  soax_status st;
  if ((st = check_rows(reinterpret_cast<const void* const*>(lamT), n, "lamT")) ||
      (st = check_rows(reinterpret_cast<const void* const*>(grad_x0), n, "grad_x0")) ||
      (st = check_abc_host(abc)))
    return st;
  if (!grad_abc) return fail(SOAX_E_ARG, "grad_abc is NULL");
  if (n < 0) return fail(SOAX_E_ARG, "bad n");
  const int64_t max_n = SOAX_ADJOINT_NOALLOC_MAX_N;
  if (n > max_n || adjoint_partials(n) * 3 * int64_t(sizeof(double)) > kNoAllocScratchBytes)
    return fail(SOAX_E_RANGE,
                "soax_adjoint_noalloc: n = %lld exceeds its fixed scratch (%lld bytes, at most "
                "%lld particles); use soax_adjoint",
                static_cast<long long>(n), static_cast<long long>(kNoAllocScratchBytes),
                static_cast<long long>(max_n));
  if (nsteps < 0 || k < 1) return fail(SOAX_E_ARG, "need nsteps >= 0 and k >= 1");
  if (!is_finite(dt)) return fail(SOAX_E_ARG, "dt is not finite");
  if (!tape && n > 0 && nsteps > 0) return fail(SOAX_E_ARG, "tape is NULL");
  double* partial = nullptr;
  if ((st = scratch_ptr(&partial))) return st;
  AdjointArgs a{};
  a.tape = tape;
  for (int d = 0; d < 3; ++d) {
    a.lam[d] = lamT[d];
    a.gx[d] = grad_x0[d];
  }
  // every partial the final sum reads is written by the adjoint kernel's
  // workgroups before it, so nothing needs clearing
  a.partial = partial;
  a.grad_abc = grad_abc;
  a.stride = 1;
  a.n = n;
  a.nsteps = nsteps;
  a.k = k;
  a.dt = dt;
  a.abc = AbcParams{abc[0], abc[1], abc[2]};
  HIP_TRY(launch_adjoint(a, as_stream(stream)), "adjoint launch");
  return SOAX_OK;
}

static soax_status sqdist_impl(const double* const* xT, int64_t stride,
                               const double* const* target, int64_t n, double* const* lamT,
                               double* loss, void* stream);

soax_status soax_sqdist_loss_strided(const double* const* xT, int64_t stride,
                                     const double* const* target, int64_t n, double* const* lamT,
                                     double* loss, void* stream) {
  soax_status st0;
  if ((st0 = check_stride(stride))) return st0;
  return sqdist_impl(xT, stride, target, n, lamT, loss, stream);
}

soax_status soax_sqdist_loss(const double* const* xT, const double* const* target, int64_t n,
                             double* const* lamT, double* loss, void* stream) {
  return sqdist_impl(xT, 1, target, n, lamT, loss, stream);
}

static soax_status sqdist_impl(const double* const* xT, int64_t stride,
                               const double* const* target, int64_t n, double* const* lamT,
                               double* loss, void* stream) {
  soax_status st;
  if ((st = check_rows(reinterpret_cast<const void* const*>(xT), n, "xT")) ||
      (st = check_rows(reinterpret_cast<const void* const*>(target), n, "target")))
    return st;
  if (lamT && (st = check_rows(reinterpret_cast<const void* const*>(lamT), n, "lamT"))) return st;
  if (!loss) return fail(SOAX_E_ARG, "loss is NULL");
  if (n < 0 || n > kMaxParticles) return fail(n < 0 ? SOAX_E_ARG : SOAX_E_RANGE, "bad n");
  hipStream_t s = as_stream(stream);
  const int64_t parts = std::max<int64_t>(loss_partials(n), 1);
  void* partial = nullptr;
  hipError_t e = hipMallocAsync(&partial, parts * 3 * sizeof(double), s);
  if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMallocAsync(partials): %s", hipGetErrorString(e));
  LossArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.xT[d] = xT[d];
    a.target[d] = target[d];
    a.lam[d] = lamT ? lamT[d] : nullptr;
  }
  a.partial = static_cast<double*>(partial);
  a.loss = loss;
  a.stride = stride;
  a.n = n;
  e = launch_sqdist_loss(a, s);
  hipError_t e2 = hipFreeAsync(partial, s);
  if (e != hipSuccess) return hip_fail(e, "loss launch");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync(partials)");
  return SOAX_OK;
}

}  // extern "C"
