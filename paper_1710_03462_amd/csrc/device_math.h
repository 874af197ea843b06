// device_math.h -- per-particle arithmetic shared by every kernel of the
// library: the periodic wrap, the ABC field and one explicit-midpoint step.
//
// Every expression is written as separate IEEE operations; the library is
// compiled with -ffp-contract=off so that x + dt*v is a multiply and an add,
// never an FMA (eq. (1) of Section 2 evaluated as written).  Only the sine
// and cosine evaluations (trig.h) use fused multiply-adds, explicitly.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"
#include "trig.h"

namespace soax {

// Periodic box edge: the double nearest to 2*pi.
constexpr double kBoxL = 6.283185307179586;

struct Abc {
  double A, B, C;
};

__device__ __forceinline__ Abc to_abc(const AbcParams& p) { return Abc{p.A, p.B, p.C}; }

// Wrap one coordinate displaced by much less than a box edge into [0, L).
// A negative coordinate whose sum with L rounds to L is stored as 0.
__device__ __forceinline__ double wrap_box(double x) {
  double lo = x + kBoxL;
  lo = (lo >= kBoxL) ? 0.0 : lo;
  double hi = x - kBoxL;
  return (x >= kBoxL) ? hi : ((x < 0.0) ? lo : x);
}

// sin and cos of the three coordinates of a point.
struct Trig3 {
  double sx, cx, sy, cy, sz, cz;
};

__device__ __forceinline__ Trig3 trig3(double x, double y, double z) {
  Trig3 t;
  trig::sincos_fast(x, &t.sx, &t.cx);
  trig::sincos_fast(y, &t.sy, &t.cy);
  trig::sincos_fast(z, &t.sz, &t.cz);
  return t;
}

// The same for the point (x + dx, y + dy, z + dz), from the values at (x, y, z).
// TIER: what the caller guarantees about every shift (trig::kTierSmall,
// kTierMid or kTierAny).
template <int TIER>
__device__ __forceinline__ Trig3 trig3_shift(const Trig3& t, double x, double y, double z,
                                             double dx, double dy, double dz) {
  Trig3 r;
  trig::sincos_shift<TIER>(x, t.sx, t.cx, dx, &r.sx, &r.cx);
  trig::sincos_shift<TIER>(y, t.sy, t.cy, dy, &r.sy, &r.cy);
  trig::sincos_shift<TIER>(z, t.sz, t.cz, dz, &r.sz, &r.cz);
  return r;
}

static_assert(kShiftLimit == trig::kShiftMax, "small_steps must match the shift bound");
static_assert(kShiftMidLimit < trig::kShiftLong, "the mid tier must stay inside the long series");
static_assert(kTierSmall == trig::kTierSmall && kTierMid == trig::kTierMid &&
                  kTierAny == trig::kTierAny,
              "shift tiers of the host and the device must agree");

// u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x), each
// component one product and one fused multiply-add
__device__ __forceinline__ void field_of(const Abc& p, const Trig3& t, double& u0, double& u1,
                                         double& u2) {
  u0 = fma(p.A, t.sz, p.C * t.cy);
  u1 = fma(p.B, t.sx, p.A * t.cz);
  u2 = fma(p.C, t.sy, p.B * t.cx);
}

__device__ __forceinline__ void abc_field(const Abc& p, double x, double y, double z, double& u0,
                                          double& u1, double& u2) {
  field_of(p, trig3(x, y, z), u0, u1, u2);
}

// One explicit-midpoint step: k1 = u(x), xm = x + (dt/2) k1, k2 = u(xm),
// x+ = x + dt k2.  On return x holds x+ (not wrapped), t the sines and
// cosines at the start point and d = dt k2 the displacement.
template <int TIER>
__device__ __forceinline__ void rk2_midpoint_parts(const Abc& p, double dt, double& x, double& y,
                                                   double& z, Trig3& t, double& d0, double& d1,
                                                   double& d2) {
  t = trig3(x, y, z);
  double k0, k1, k2;
  field_of(p, t, k0, k1, k2);
  const double h = 0.5 * dt;
  const Trig3 tm = trig3_shift<TIER>(t, x, y, z, h * k0, h * k1, h * k2);
  field_of(p, tm, k0, k1, k2);
  d0 = dt * k0;
  d1 = dt * k1;
  d2 = dt * k2;
  x = x + d0;
  y = y + d1;
  z = z + d2;
}

// The field's amplitudes times s: s u(x) is then one product and one fma
// per component, like u(x) itself.
__device__ __forceinline__ Abc scaled(const Abc& p, double s) {
  return Abc{s * p.A, s * p.B, s * p.C};
}

// Alignment (bytes) of a run of VEC consecutive T starting at a multiple of
// VEC elements in a 16-byte aligned array.
template <typename T, int VEC>
__device__ constexpr size_t run_align() {
  return sizeof(T) * VEC < 16 ? sizeof(T) * VEC : 16;
}

// Vector of VEC elements of T (VEC = 1: T itself).
template <typename T, int VEC>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(VEC)));
};
template <typename T>
struct VecOf<T, 1> {
  typedef T type;
};

// A run of VEC consecutive elements moved as chunks of at most 16 bytes.
// NT: nontemporal hint, for streams that are not touched again soon: large
// read-only inputs and every output of a step whose data far exceeds the
// caches (measured on the MI355X: an in-place Euler step at 1e8 particles
// goes from 5.3 to 6.4 TB/s with nontemporal velocity loads and stores).
template <typename T, int VEC>
struct RunChunk {
  static constexpr int kBytes = sizeof(T) * VEC < 16 ? static_cast<int>(sizeof(T)) * VEC : 16;
  static constexpr int kElems = kBytes / static_cast<int>(sizeof(T));
  static constexpr int kChunks = VEC / kElems;
  using V = typename VecOf<T, kElems>::type;
};

template <bool NT, typename T, int VEC>
__device__ __forceinline__ void ld_run(const T* p, T (&v)[VEC]) {
  using C = RunChunk<T, VEC>;
#pragma unroll
  for (int c = 0; c < C::kChunks; ++c) {
    const typename C::V* q = reinterpret_cast<const typename C::V*>(p + c * C::kElems);
    typename C::V t;
    if constexpr (NT)
      t = __builtin_nontemporal_load(q);
    else
      t = *q;
    __builtin_memcpy(&v[c * C::kElems], &t, C::kBytes);
  }
}

template <bool NT, typename T, int VEC>
__device__ __forceinline__ void st_run(T* p, const T (&v)[VEC]) {
  using C = RunChunk<T, VEC>;
#pragma unroll
  for (int c = 0; c < C::kChunks; ++c) {
    typename C::V* q = reinterpret_cast<typename C::V*>(p + c * C::kElems);
    typename C::V t;
    __builtin_memcpy(&t, &v[c * C::kElems], C::kBytes);
    if constexpr (NT)
      __builtin_nontemporal_store(t, q);
    else
      *q = t;
  }
}

template <bool NT, typename T>
__device__ __forceinline__ T ld1(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st1(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ------------------------------------------------ streaming through buffers
//
// The streaming kernels address each array through a buffer resource that
// covers one workgroup's run of elements, because buffer loads and stores
// carry the full set of gfx950 cache-policy bits (bit 0 sc0, bit 1 nt,
// bit 4 sc1), where plain global accesses reach only nt.  Loads are nt (the
// data is not reused); stores are nt at system scope (sc0 sc1 nt), which
// writes them through without keeping them in the caches.  Measured at 1e8
// particles against nt loads and stores through global pointers: Euler step
// 0.91 -> 0.88 ms, RK2 step 1.05 -> 1.02 ms.  The offsets are 32-bit and
// small (one workgroup's run), and every access is in range: the kernels
// take the buffer path only for whole runs.
constexpr int kPolicyLoadStream = 2;    // nt
constexpr int kPolicyStoreStream = 19;  // sc0 | nt | sc1
// Word 3 of an unformatted buffer resource on the gfx9 family.
constexpr int kRsrcWord3 = 0x00020000;

template <typename T>
struct Window {
  __amdgpu_buffer_rsrc_t r;
};

// count elements of base starting at element first (count * sizeof(T) < 2^31)
template <typename T>
__device__ __forceinline__ Window<T> window(const T* base, int64_t first, int64_t count) {
  return Window<T>{__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base) + first, 0,
                                                     static_cast<int>(count * sizeof(T)),
                                                     kRsrcWord3)};
}

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

template <int BYTES>
struct RawChunk;
template <>
struct RawChunk<4> {
  using V = unsigned int;
  __device__ static V ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kPolicyLoadStream);
  }
  __device__ static void st(V v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, kPolicyStoreStream);
  }
};
template <>
struct RawChunk<8> {
  using V = u32x2_t;
  __device__ static V ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kPolicyLoadStream);
  }
  __device__ static void st(V v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, kPolicyStoreStream);
  }
};
template <>
struct RawChunk<16> {
  using V = u32x4_t;
  __device__ static V ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kPolicyLoadStream);
  }
  __device__ static void st(V v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kPolicyStoreStream);
  }
};

// VEC consecutive elements from element e of the window, as chunks of at most
// 16 bytes (the same chunking as ld_run / st_run).
template <typename T, int VEC>
__device__ __forceinline__ void win_ld_run(Window<T> w, int e, T (&v)[VEC]) {
  using C = RunChunk<T, VEC>;
  using R = RawChunk<C::kBytes>;
#pragma unroll
  for (int c = 0; c < C::kChunks; ++c) {
    const typename R::V t = R::ld(w.r, (e + c * C::kElems) * static_cast<int>(sizeof(T)));
    __builtin_memcpy(&v[c * C::kElems], &t, C::kBytes);
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void win_st_run(Window<T> w, int e, const T (&v)[VEC]) {
  using C = RunChunk<T, VEC>;
  using R = RawChunk<C::kBytes>;
#pragma unroll
  for (int c = 0; c < C::kChunks; ++c) {
    typename R::V t;
    __builtin_memcpy(&t, &v[c * C::kElems], C::kBytes);
    R::st(t, w.r, (e + c * C::kElems) * static_cast<int>(sizeof(T)));
  }
}

template <typename T>
__device__ __forceinline__ T win_ld1(Window<T> w, int e) {
  T v[1];
  win_ld_run<T, 1>(w, e, v);
  return v[0];
}

template <typename T>
__device__ __forceinline__ void win_st1(Window<T> w, int e, T x) {
  const T v[1] = {x};
  win_st_run<T, 1>(w, e, v);
}

template <typename T>
__device__ __forceinline__ double widen(T v) {
  return static_cast<double>(v);
}

// One component of an Euler step (eq. (1)): the new position, and for
// EULER_ACC the new velocity from the acceleration.  The same arithmetic as
// update_particle, one coordinate at a time.
template <int INTEG, typename PT, typename VT>
__device__ __forceinline__ void euler_component(PT& x, VT& v, VT a, double dt, int wrap) {
  // symplectic Euler: the velocity first, rounded to its type, then the
  // position with the new velocity
  if constexpr (INTEG == kSymEuler) v = static_cast<VT>(widen(v) + dt * widen(a));
  double y = widen(x) + dt * widen(v);
  if constexpr (std::is_same<PT, double>::value) {
    if (wrap) y = wrap_box(y);
  }
  x = static_cast<PT>(y);
  if constexpr (INTEG == kEulerAcc) v = static_cast<VT>(widen(v) + dt * widen(a));
}

// One Heun step (explicit trapezoid): k1 = u(x), k2 = u(x + dt k1),
// d = (dt/2)(k1 + k2); t holds the start point's sines and cosines.
template <int TIER>
__device__ __forceinline__ void heun_parts(const Abc& p, double dt, double x, double y, double z,
                                           Trig3& t, double& d0, double& d1, double& d2) {
  t = trig3(x, y, z);
  double a0, a1, a2, b0, b1, b2;
  field_of(p, t, a0, a1, a2);
  field_of(p, trig3_shift<TIER>(t, x, y, z, dt * a0, dt * a1, dt * a2), b0, b1, b2);
  const double h = 0.5 * dt;
  d0 = h * (a0 + b0);
  d1 = h * (a1 + b1);
  d2 = h * (a2 + b2);
}

// One classical RK4 step: k1 = u(x), k2 = u(x + dt/2 k1), k3 = u(x + dt/2 k2),
// k4 = u(x + dt k3), d = dt/6 (k1 + 2 k2 + 2 k3 + k4); every stage's sines come
// from the start point's by angle addition.
template <int TIER>
__device__ __forceinline__ void rk4_parts(const Abc& p, double dt, double x, double y, double z,
                                          Trig3& t, double& d0, double& d1, double& d2) {
  t = trig3(x, y, z);
  const double h = 0.5 * dt;
  double k10, k11, k12, k20, k21, k22, k30, k31, k32, k40, k41, k42;
  field_of(p, t, k10, k11, k12);
  field_of(p, trig3_shift<TIER>(t, x, y, z, h * k10, h * k11, h * k12), k20, k21, k22);
  field_of(p, trig3_shift<TIER>(t, x, y, z, h * k20, h * k21, h * k22), k30, k31, k32);
  field_of(p, trig3_shift<TIER>(t, x, y, z, dt * k30, dt * k31, dt * k32), k40, k41, k42);
  const double s = dt / 6.0;
  d0 = s * (k10 + 2.0 * k20 + 2.0 * k30 + k40);
  d1 = s * (k11 + 2.0 * k21 + 2.0 * k31 + k41);
  d2 = s * (k12 + 2.0 * k22 + 2.0 * k32 + k42);
}

// The positions (y0, y1, y2) one step of a field integrator after
// (s0, s1, s2), not wrapped; t: the start point's sines and cosines, d: the
// displacement, from which the field at the new position follows by angle
// addition.
template <int INTEG, int TIER>
__device__ __forceinline__ void field_step(const Abc& p, double dt, double s0, double s1,
                                           double s2, double& y0, double& y1, double& y2,
                                           Trig3& t, double& d0, double& d1, double& d2) {
  if constexpr (INTEG == kRk2Abc) {
    y0 = s0;
    y1 = s1;
    y2 = s2;
    rk2_midpoint_parts<TIER>(p, dt, y0, y1, y2, t, d0, d1, d2);
  } else {
    if constexpr (INTEG == kHeunAbc) heun_parts<TIER>(p, dt, s0, s1, s2, t, d0, d1, d2);
    else rk4_parts<TIER>(p, dt, s0, s1, s2, t, d0, d1, d2);
    y0 = s0 + d0;
    y1 = s1 + d1;
    y2 = s2 + d2;
  }
}

// Advance one particle.  Positions and velocities are widened to double,
// combined in double and rounded back on store.  TIER: shift_tier of the
// step (field integrators only; the results do not depend on it).
template <int INTEG, typename PT, typename VT, int TIER>
__device__ __forceinline__ void update_particle(PT& x0, PT& x1, PT& x2, VT& v0, VT& v1, VT& v2,
                                                VT a0, VT a1, VT a2, double dt, const Abc& p,
                                                int wrap) {
  if constexpr (INTEG == kSymEuler) {
    euler_component<INTEG, PT, VT>(x0, v0, a0, dt, wrap);
    euler_component<INTEG, PT, VT>(x1, v1, a1, dt, wrap);
    euler_component<INTEG, PT, VT>(x2, v2, a2, dt, wrap);
  } else if constexpr (INTEG == kEuler || INTEG == kEulerAcc) {
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
    const double s0 = widen(x0), s1 = widen(x1), s2 = widen(x2);
    double y0, y1, y2;
    Trig3 t;
    double d0, d1, d2;
    field_step<INTEG, TIER>(p, dt, s0, s1, s2, y0, y1, y2, t, d0, d1, d2);
    if (wrap) {
      y0 = wrap_box(y0);
      y1 = wrap_box(y1);
      y2 = wrap_box(y2);
    }
    x0 = static_cast<PT>(y0);
    x1 = static_cast<PT>(y1);
    x2 = static_cast<PT>(y2);
    // the stored velocity is the field at the new position (the field is
    // 2pi-periodic, so the shift from the start point needs no wrap)
    double u0, u1, u2;
    field_of(p, trig3_shift<TIER>(t, s0, s1, s2, d0, d1, d2), u0, u1, u2);
    v0 = static_cast<VT>(u0);
    v1 = static_cast<VT>(u1);
    v2 = static_cast<VT>(u2);
  }
}

}  // namespace soax
