// device_math.h -- per-particle arithmetic shared by every kernel of the
// library: the periodic wrap, the ABC field and one explicit-midpoint step.
//
// Every expression is written as separate IEEE operations; the library is
// compiled with -ffp-contract=off so that x + dt*v is a multiply and an add,
// never an FMA (eq. (1) of Section 2 evaluated as written).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"

namespace soax {

// Periodic box edge: the double nearest to 2*pi.
constexpr double kBoxL = 6.283185307179586;

struct Abc {
  double A, B, C;
};

// Wrap one coordinate displaced by much less than a box edge into [0, L).
// A negative coordinate whose sum with L rounds to L is stored as 0.
__device__ __forceinline__ double wrap_box(double x) {
  double lo = x + kBoxL;
  lo = (lo >= kBoxL) ? 0.0 : lo;
  double hi = x - kBoxL;
  return (x >= kBoxL) ? hi : ((x < 0.0) ? lo : x);
}

// sin and cos of one fp64 argument (ROCm device math library).
__device__ __forceinline__ void sincos_f64(double x, double* s, double* c) { sincos(x, s, c); }

// u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)
__device__ __forceinline__ void abc_field(const Abc& p, double x, double y, double z, double& u0,
                                          double& u1, double& u2) {
  double sx, cx, sy, cy, sz, cz;
  sincos_f64(x, &sx, &cx);
  sincos_f64(y, &sy, &cy);
  sincos_f64(z, &sz, &cz);
  u0 = p.A * sz + p.C * cy;
  u1 = p.B * sx + p.A * cz;
  u2 = p.C * sy + p.B * cx;
}

// One explicit-midpoint step without wrap: k1 = u(x), xm = x + (dt/2) k1,
// x <- x + dt u(xm).
__device__ __forceinline__ void rk2_midpoint(const Abc& p, double dt, double& x, double& y,
                                             double& z) {
  double k0, k1, k2;
  abc_field(p, x, y, z, k0, k1, k2);
  const double h = 0.5 * dt;
  const double xm = x + h * k0, ym = y + h * k1, zm = z + h * k2;
  abc_field(p, xm, ym, zm, k0, k1, k2);
  x = x + dt * k0;
  y = y + dt * k1;
  z = z + dt * k2;
}

// Alignment (bytes) of a run of VEC consecutive T starting at a multiple of
// VEC elements in a 16-byte aligned array.
template <typename T, int VEC>
__device__ constexpr size_t run_align() {
  return sizeof(T) * VEC < 16 ? sizeof(T) * VEC : 16;
}

__device__ __forceinline__ Abc to_abc(const AbcParams& p) { return Abc{p.A, p.B, p.C}; }

template <typename T>
__device__ __forceinline__ double widen(T v) {
  return static_cast<double>(v);
}

// Advance one particle.  Positions and velocities are widened to double,
// combined in double and rounded back on store.
template <int INTEG, typename PT, typename VT>
__device__ __forceinline__ void update_particle(PT& x0, PT& x1, PT& x2, VT& v0, VT& v1, VT& v2,
                                                VT a0, VT a1, VT a2, double dt, const Abc& p,
                                                int wrap) {
  if constexpr (INTEG == kEuler || INTEG == kEulerAcc) {
    double y0 = widen(x0) + dt * widen(v0);
    double y1 = widen(x1) + dt * widen(v1);
    double y2 = widen(x2) + dt * widen(v2);
    if constexpr (std::is_same<PT, double>::value) {
      if (wrap) {
        y0 = wrap_box(y0);
        y1 = wrap_box(y1);
        y2 = wrap_box(y2);
      }
    }
    x0 = static_cast<PT>(y0);
    x1 = static_cast<PT>(y1);
    x2 = static_cast<PT>(y2);
    if constexpr (INTEG == kEulerAcc) {
      v0 = static_cast<VT>(widen(v0) + dt * widen(a0));
      v1 = static_cast<VT>(widen(v1) + dt * widen(a1));
      v2 = static_cast<VT>(widen(v2) + dt * widen(a2));
    }
  } else {
    double y0 = widen(x0), y1 = widen(x1), y2 = widen(x2);
    rk2_midpoint(p, dt, y0, y1, y2);
    if (wrap) {
      y0 = wrap_box(y0);
      y1 = wrap_box(y1);
      y2 = wrap_box(y2);
    }
    x0 = static_cast<PT>(y0);
    x1 = static_cast<PT>(y1);
    x2 = static_cast<PT>(y2);
    double u0, u1, u2;
    abc_field(p, y0, y1, y2, u0, u1, u2);
    v0 = static_cast<VT>(u0);
    v1 = static_cast<VT>(u1);
    v2 = static_cast<VT>(u2);
  }
}

}  // namespace soax
