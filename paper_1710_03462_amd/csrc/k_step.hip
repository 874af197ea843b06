// k_step.hip -- gfx950 kernels for the per-particle time step in both
// layouts, the bulk AoS<->SoA transposes, the seeded fill and the copy probe.
//
// The step (Section 2, eq. (1) and its RK2 / acceleration variants) is a
// streaming read-modify-write with no reuse inside a step, so the kernels are
// shaped for HBM, not for the matrix cores:
//  * SoA: each thread owns `VEC` consecutive particles (one by default; two,
//    with 16-byte position accesses, for the field integrators on sets that
//    stream from HBM, where that shape measured fastest), so a wave reads and
//    writes each array it touches as one contiguous run; arrays the step does
//    not use (id, mass, ...) are never read, the SoA advantage of Section 2.
//  * AoS: a workgroup stages a tile of whole records through LDS with
//    coalesced 16-byte accesses, updates the records in LDS and writes the
//    tile back, so the only waste is the bytes of unused fields, not the
//    uncoalesced pattern of Section 3.2; the naive kernel keeps that pattern
//    (one thread per record, direct per-field accesses) for comparison.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device_math.h"
#include "launch.h"

namespace soax {

namespace {

constexpr int kLdsBudget = 48 * 1024;  // bytes of LDS staging per workgroup



// ------------------------------------------------------------ SoA step

// Loads and stores of the SoA step.  STREAM (the step's arrays far exceed
// the caches): through buffer windows over this workgroup's run of
// particles, nt loads and write-through nt stores; otherwise ordinary global
// accesses.  first / cnt: the workgroup's run, e: the thread's first element
// in it.
template <bool STREAM, typename T, int VEC>
__device__ __forceinline__ void step_ld(const T* base, int64_t first, int64_t cnt, int e,
                                        T (&v)[VEC]) {
  if constexpr (STREAM) win_ld_run<T, VEC>(window(base, first, cnt), e, v);
  else ld_run<false, T, VEC>(base + first + e, v);
}

template <bool STREAM, typename T, int VEC>
__device__ __forceinline__ void step_st(T* base, int64_t first, int64_t cnt, int e,
                                        const T (&v)[VEC]) {
  if constexpr (STREAM) win_st_run<T, VEC>(window(base, first, cnt), e, v);
  else st_run<false, T, VEC>(base + first + e, v);
}

template <int INTEG, typename PT, typename VT, int VEC, int TIER, bool STREAM>
__global__ __launch_bounds__(1024) void soa_step_kernel(SoaStepArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t i0 = t * VEC;
  if (i0 >= a.n) return;
  const Abc p = to_abc(a.abc);
  PT* px = static_cast<PT*>(a.pos[0]);
  PT* py = static_cast<PT*>(a.pos[1]);
  PT* pz = static_cast<PT*>(a.pos[2]);
  VT* vx = static_cast<VT*>(a.vel[0]);
  VT* vy = static_cast<VT*>(a.vel[1]);
  VT* vz = static_cast<VT*>(a.vel[2]);
  const VT* ax = static_cast<const VT*>(a.acc[0]);
  const VT* ay = static_cast<const VT*>(a.acc[1]);
  const VT* az = static_cast<const VT*>(a.acc[2]);
  constexpr bool kReadsVel = !field_integrator(INTEG);  // field steps overwrite vel unread
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x * VEC;
  const int64_t cnt = min(static_cast<int64_t>(blockDim.x) * VEC, a.n - first);
  const int e = static_cast<int>(threadIdx.x) * VEC;

  if constexpr (!field_integrator(INTEG) && STREAM) {
    if (i0 + VEC <= a.n) {
      // Streaming Euler steps are independent per coordinate: one component
      // at a time (its loads, update and stores) keeps two or three streams
      // per wave in flight instead of six -- faster on HBM for this in-place
      // update.  Cache-resident sets take the path below, whose loads all
      // leave before the first store: there the step is bound by latency,
      // and the component order waits out three round trips in turn (its
      // kernel took 2.4-2.5 us at 1e3 particles against 2.2 us).
      PT* P[3] = {px, py, pz};
      VT* Vv[3] = {vx, vy, vz};
      const VT* G[3] = {ax, ay, az};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        PT x[VEC];
        VT v[VEC], g[VEC];
        step_ld<true, PT, VEC>(P[d], first, cnt, e, x);
        step_ld<true, VT, VEC>(Vv[d], first, cnt, e, v);
        if constexpr (uses_acc(INTEG)) step_ld<true, VT, VEC>(G[d], first, cnt, e, g);
#pragma unroll
        for (int j = 0; j < VEC; ++j)
          euler_component<INTEG, PT, VT>(x[j], v[j], uses_acc(INTEG) ? g[j] : VT(0), a.dt,
                                         a.wrap);
        step_st<true, PT, VEC>(P[d], first, cnt, e, x);
        if constexpr (uses_acc(INTEG)) step_st<true, VT, VEC>(Vv[d], first, cnt, e, v);
      }
      return;
    }
  }
  if (i0 + VEC <= a.n) {
    PT x[VEC], y[VEC], z[VEC];
    VT u[VEC], v[VEC], w[VEC];
    VT ga[VEC], gb[VEC], gc[VEC];
    step_ld<STREAM, PT, VEC>(px, first, cnt, e, x);
    step_ld<STREAM, PT, VEC>(py, first, cnt, e, y);
    step_ld<STREAM, PT, VEC>(pz, first, cnt, e, z);
    if constexpr (kReadsVel) {
      step_ld<STREAM, VT, VEC>(vx, first, cnt, e, u);
      step_ld<STREAM, VT, VEC>(vy, first, cnt, e, v);
      step_ld<STREAM, VT, VEC>(vz, first, cnt, e, w);
    }
    if constexpr (uses_acc(INTEG)) {
      step_ld<STREAM, VT, VEC>(ax, first, cnt, e, ga);
      step_ld<STREAM, VT, VEC>(ay, first, cnt, e, gb);
      step_ld<STREAM, VT, VEC>(az, first, cnt, e, gc);
    } else {
#pragma unroll
      for (int j = 0; j < VEC; ++j) ga[j] = gb[j] = gc[j] = VT(0);
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
      if constexpr (!kReadsVel) u[j] = v[j] = w[j] = VT(0);
      update_particle<INTEG, PT, VT, TIER>(x[j], y[j], z[j], u[j], v[j], w[j], ga[j], gb[j],
                                            gc[j], a.dt, p, a.wrap);
    }
    step_st<STREAM, PT, VEC>(px, first, cnt, e, x);
    step_st<STREAM, PT, VEC>(py, first, cnt, e, y);
    step_st<STREAM, PT, VEC>(pz, first, cnt, e, z);
    if constexpr (INTEG != kEuler) {
      step_st<STREAM, VT, VEC>(vx, first, cnt, e, u);
      step_st<STREAM, VT, VEC>(vy, first, cnt, e, v);
      step_st<STREAM, VT, VEC>(vz, first, cnt, e, w);
    }
  } else {
    for (int64_t i = i0; i < a.n; ++i) {
      PT x = px[i], y = py[i], z = pz[i];
      VT u = kReadsVel ? vx[i] : VT(0), v = kReadsVel ? vy[i] : VT(0),
         w = kReadsVel ? vz[i] : VT(0);
      VT g0 = VT(0), g1 = VT(0), g2 = VT(0);
      if constexpr (uses_acc(INTEG)) {
        g0 = ax[i];
        g1 = ay[i];
        g2 = az[i];
      }
      update_particle<INTEG, PT, VT, TIER>(x, y, z, u, v, w, g0, g1, g2, a.dt, p, a.wrap);
      px[i] = x;
      py[i] = y;
      pz[i] = z;
      if constexpr (INTEG != kEuler) {
        vx[i] = u;
        vy[i] = v;
        vz[i] = w;
      }
    }
  }
}

// The RK4 step on streaming sets.  Each workgroup takes two consecutive runs
// of blockDim.x * VEC particles and issues the second run's position loads
// before the first run's arithmetic, so that they are in flight while it
// computes.  RK4 issues 1.6x the fp64 instructions of RK2 and its arithmetic and memory
// traffic overlap less; this order made it about 3% faster at 1e8 particles
// (1.28 against 1.32 ms, interleaved runs), while it made RK2 and Heun no
// faster.  The last, incomplete pair of runs is stepped one particle per
// thread with the same arithmetic, so the results do not depend on the
// shape.
template <typename PT, typename VT, int VEC, int TIER>
__global__ __launch_bounds__(1024) void soa_rk4_two_runs_kernel(SoaStepArgs a) {
  const Abc p = to_abc(a.abc);
  PT* px = static_cast<PT*>(a.pos[0]);
  PT* py = static_cast<PT*>(a.pos[1]);
  PT* pz = static_cast<PT*>(a.pos[2]);
  VT* vx = static_cast<VT*>(a.vel[0]);
  VT* vy = static_cast<VT*>(a.vel[1]);
  VT* vz = static_cast<VT*>(a.vel[2]);
  const int64_t run = static_cast<int64_t>(blockDim.x) * VEC;
  const int64_t fa = static_cast<int64_t>(blockIdx.x) * 2 * run;
  const int64_t fb = fa + run;
  const int e = static_cast<int>(threadIdx.x) * VEC;
  if (fb + run <= a.n) {
    PT xa[VEC], ya[VEC], za[VEC], xb[VEC], yb[VEC], zb[VEC];
    step_ld<true, PT, VEC>(px, fa, run, e, xa);
    step_ld<true, PT, VEC>(py, fa, run, e, ya);
    step_ld<true, PT, VEC>(pz, fa, run, e, za);
    step_ld<true, PT, VEC>(px, fb, run, e, xb);
    step_ld<true, PT, VEC>(py, fb, run, e, yb);
    step_ld<true, PT, VEC>(pz, fb, run, e, zb);
    VT u[VEC], v[VEC], w[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
      u[j] = v[j] = w[j] = VT(0);
      update_particle<kRk4Abc, PT, VT, TIER>(xa[j], ya[j], za[j], u[j], v[j], w[j], VT(0), VT(0),
                                             VT(0), a.dt, p, a.wrap);
    }
    step_st<true, PT, VEC>(px, fa, run, e, xa);
    step_st<true, PT, VEC>(py, fa, run, e, ya);
    step_st<true, PT, VEC>(pz, fa, run, e, za);
    step_st<true, VT, VEC>(vx, fa, run, e, u);
    step_st<true, VT, VEC>(vy, fa, run, e, v);
    step_st<true, VT, VEC>(vz, fa, run, e, w);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
      u[j] = v[j] = w[j] = VT(0);
      update_particle<kRk4Abc, PT, VT, TIER>(xb[j], yb[j], zb[j], u[j], v[j], w[j], VT(0), VT(0),
                                             VT(0), a.dt, p, a.wrap);
    }
    step_st<true, PT, VEC>(px, fb, run, e, xb);
    step_st<true, PT, VEC>(py, fb, run, e, yb);
    step_st<true, PT, VEC>(pz, fb, run, e, zb);
    step_st<true, VT, VEC>(vx, fb, run, e, u);
    step_st<true, VT, VEC>(vy, fb, run, e, v);
    step_st<true, VT, VEC>(vz, fb, run, e, w);
    return;
  }
  const int64_t end = min(fa + 2 * run, a.n);
  for (int64_t i = fa + threadIdx.x; i < end; i += blockDim.x) {
    PT x = px[i], y = py[i], z = pz[i];
    VT u = VT(0), v = VT(0), w = VT(0);
    update_particle<kRk4Abc, PT, VT, TIER>(x, y, z, u, v, w, VT(0), VT(0), VT(0), a.dt, p,
                                           a.wrap);
    px[i] = x;
    py[i] = y;
    pz[i] = z;
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
  }
}

template <int INTEG, typename PT, typename VT, int TIER, bool STREAM>
hipError_t soa_step_launch(int vec, int64_t grid, int block, const SoaStepArgs& a, hipStream_t s) {
  if constexpr (INTEG == kRk4Abc && STREAM) {
    // grid counts runs of block * vec particles; one workgroup per two runs
    const int64_t pairs = (grid + 1) / 2;
    if (vec == 1)
      hipLaunchKernelGGL((soa_rk4_two_runs_kernel<PT, VT, 1, TIER>), dim3(pairs), dim3(block), 0,
                         s, a);
    else
      hipLaunchKernelGGL((soa_rk4_two_runs_kernel<PT, VT, 2, TIER>), dim3(pairs), dim3(block), 0,
                         s, a);
    return hipGetLastError();
  }
  if constexpr (INTEG == kHeunAbc || INTEG == kRk4Abc) {
    // one or two particles per thread (the host caps vec at 2 for these)
    if (vec == 1)
      hipLaunchKernelGGL((soa_step_kernel<INTEG, PT, VT, 1, TIER, STREAM>), dim3(grid),
                         dim3(block), 0, s, a);
    else
      hipLaunchKernelGGL((soa_step_kernel<INTEG, PT, VT, 2, TIER, STREAM>), dim3(grid),
                         dim3(block), 0, s, a);
    return hipGetLastError();
  }
  switch (vec) {
    case 1:
      hipLaunchKernelGGL((soa_step_kernel<INTEG, PT, VT, 1, TIER, STREAM>), dim3(grid),
                         dim3(block), 0, s, a);
      break;
    case 2:
      hipLaunchKernelGGL((soa_step_kernel<INTEG, PT, VT, 2, TIER, STREAM>), dim3(grid),
                         dim3(block), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((soa_step_kernel<INTEG, PT, VT, 4, TIER, STREAM>), dim3(grid),
                         dim3(block), 0, s, a);
      break;
  }
  return hipGetLastError();
}

template <int INTEG, typename PT, typename VT, int TIER>
hipError_t soa_step_stream(bool stream, int vec, int64_t grid, int block, const SoaStepArgs& a,
                           hipStream_t s) {
  return stream ? soa_step_launch<INTEG, PT, VT, TIER, true>(vec, grid, block, a, s)
                : soa_step_launch<INTEG, PT, VT, TIER, false>(vec, grid, block, a, s);
}

template <int INTEG, typename PT, typename VT>
hipError_t soa_step_vec(int vec, int block, const SoaStepArgs& a, hipStream_t s) {
  if constexpr (INTEG == kHeunAbc || INTEG == kRk4Abc) vec = vec > 2 ? 2 : vec;
  const int64_t threads = (a.n + vec - 1) / vec;
  const int64_t grid = (threads + block - 1) / block;
  if (grid == 0) return hipSuccess;
  const int64_t bytes = soa_step_bytes(INTEG, sizeof(PT), sizeof(VT));
  const bool stream = a.n * bytes >= kStreamBytes;
  if constexpr (field_integrator(INTEG)) {
    const int tier = shift_tier(a.dt, a.abc.A, a.abc.B, a.abc.C);
    if (tier == kTierSmall)
      return soa_step_stream<INTEG, PT, VT, kTierSmall>(stream, vec, grid, block, a, s);
    if (tier == kTierMid)
      return soa_step_stream<INTEG, PT, VT, kTierMid>(stream, vec, grid, block, a, s);
  }
  return soa_step_stream<INTEG, PT, VT, kTierAny>(stream, vec, grid, block, a, s);
}

// ---------------------------------------------------------- fused steps

// nsteps steps of one particle per thread with the particle held in registers
// in between: the arrays are read and written once per launch instead of once
// per step.  Each step is the arithmetic of update_particle, so the results
// equal nsteps launches of the one-step kernels bit for bit; for the field
// integrators the velocity, which no step reads, is evaluated once, at the
// final position, from the last step's sines, cosines and displacement.
template <int INTEG, typename PT, typename VT, int TIER>
__global__ __launch_bounds__(256) void soa_fused_kernel(SoaStepArgs a, int64_t nsteps) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Abc p = to_abc(a.abc);
  PT* px = static_cast<PT*>(a.pos[0]);
  PT* py = static_cast<PT*>(a.pos[1]);
  PT* pz = static_cast<PT*>(a.pos[2]);
  VT* vx = static_cast<VT*>(a.vel[0]);
  VT* vy = static_cast<VT*>(a.vel[1]);
  VT* vz = static_cast<VT*>(a.vel[2]);
  PT x = px[i], y = py[i], z = pz[i];
  if constexpr (field_integrator(INTEG)) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    Trig3 t{};
    for (int64_t k = 0; k < nsteps; ++k) {
      s0 = x;
      s1 = y;
      s2 = z;
      double y0, y1, y2;
      field_step<INTEG, TIER>(p, a.dt, s0, s1, s2, y0, y1, y2, t, d0, d1, d2);
      if (a.wrap) {
        y0 = wrap_box(y0);
        y1 = wrap_box(y1);
        y2 = wrap_box(y2);
      }
      x = y0;
      y = y1;
      z = y2;
    }
    double u0, u1, u2;
    field_of(p, trig3_shift<TIER>(t, s0, s1, s2, d0, d1, d2), u0, u1, u2);
    vx[i] = static_cast<VT>(u0);
    vy[i] = static_cast<VT>(u1);
    vz[i] = static_cast<VT>(u2);
  } else {
    VT u = vx[i], v = vy[i], w = vz[i];
    VT g0 = VT(0), g1 = VT(0), g2 = VT(0);
    if constexpr (uses_acc(INTEG)) {
      g0 = static_cast<const VT*>(a.acc[0])[i];
      g1 = static_cast<const VT*>(a.acc[1])[i];
      g2 = static_cast<const VT*>(a.acc[2])[i];
    }
    for (int64_t k = 0; k < nsteps; ++k)
      update_particle<INTEG, PT, VT, kTierAny>(x, y, z, u, v, w, g0, g1, g2, a.dt, p, a.wrap);
    if constexpr (INTEG != kEuler) {
      vx[i] = u;
      vy[i] = v;
      vz[i] = w;
    }
  }
  px[i] = x;
  py[i] = y;
  pz[i] = z;
}

template <int INTEG, typename PT, typename VT>
hipError_t soa_fused_launch(int block, const SoaStepArgs& a, int64_t nsteps, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  if (grid == 0 || nsteps <= 0) return hipSuccess;
  int tier = kTierAny;
  if constexpr (field_integrator(INTEG)) tier = shift_tier(a.dt, a.abc.A, a.abc.B, a.abc.C);
  if (tier == kTierSmall)
    hipLaunchKernelGGL((soa_fused_kernel<INTEG, PT, VT, kTierSmall>), dim3(grid), dim3(block), 0,
                       s, a, nsteps);
  else if (tier == kTierMid)
    hipLaunchKernelGGL((soa_fused_kernel<INTEG, PT, VT, kTierMid>), dim3(grid), dim3(block), 0,
                       s, a, nsteps);
  else
    hipLaunchKernelGGL((soa_fused_kernel<INTEG, PT, VT, kTierAny>), dim3(grid), dim3(block), 0,
                       s, a, nsteps);
  return hipGetLastError();
}

// ------------------------------------------------------- AoS element access

template <typename T, bool ALIGNED>
__device__ __forceinline__ T rec_load(const char* p) {
  if constexpr (ALIGNED) {
    return *reinterpret_cast<const T*>(p);
  } else {
    T v;
    __builtin_memcpy(&v, p, sizeof(T));
    return v;
  }
}

template <typename T, bool ALIGNED>
__device__ __forceinline__ void rec_store(char* p, T v) {
  if constexpr (ALIGNED) {
    *reinterpret_cast<T*>(p) = v;
  } else {
    __builtin_memcpy(p, &v, sizeof(T));
  }
}

// Update the record at `rec` (in LDS or global memory) in place.
template <int INTEG, typename PT, typename VT, bool ALIGNED, int TIER>
__device__ __forceinline__ void update_record(char* rec, const AosStepArgs& a, const Abc& p) {
  char* P = rec + a.off_pos;
  char* V = rec + a.off_vel;
  PT x = rec_load<PT, ALIGNED>(P), y = rec_load<PT, ALIGNED>(P + sizeof(PT)),
     z = rec_load<PT, ALIGNED>(P + 2 * sizeof(PT));
  VT u = VT(0), v = VT(0), w = VT(0), g0 = VT(0), g1 = VT(0), g2 = VT(0);
  if constexpr (!field_integrator(INTEG)) {
    u = rec_load<VT, ALIGNED>(V);
    v = rec_load<VT, ALIGNED>(V + sizeof(VT));
    w = rec_load<VT, ALIGNED>(V + 2 * sizeof(VT));
  }
  if constexpr (uses_acc(INTEG)) {
    const char* G = rec + a.off_acc;
    g0 = rec_load<VT, ALIGNED>(G);
    g1 = rec_load<VT, ALIGNED>(G + sizeof(VT));
    g2 = rec_load<VT, ALIGNED>(G + 2 * sizeof(VT));
  }
  update_particle<INTEG, PT, VT, TIER>(x, y, z, u, v, w, g0, g1, g2, a.dt, p, a.wrap);
  rec_store<PT, ALIGNED>(P, x);
  rec_store<PT, ALIGNED>(P + sizeof(PT), y);
  rec_store<PT, ALIGNED>(P + 2 * sizeof(PT), z);
  if constexpr (INTEG != kEuler) {
    rec_store<VT, ALIGNED>(V, u);
    rec_store<VT, ALIGNED>(V + sizeof(VT), v);
    rec_store<VT, ALIGNED>(V + 2 * sizeof(VT), w);
  }
}

// Copy `nbytes` from global `g` (16-byte aligned) into LDS with 16-byte
// accesses, consecutive lanes on consecutive chunks; the remainder bytewise.
// STREAM: the 16-byte chunks go through a buffer window over the tile with the
// streaming cache policies (see Window).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each thread issues up to kStageLoads chunk loads before it writes any of
// them to LDS, so a wave keeps several requests in flight instead of waiting
// on one chunk at a time.
constexpr int kStageLoads = 4;

template <bool STREAM>
__device__ __forceinline__ void stage_in(char* lds, const char* g, int nbytes) {
  const int nchunk = nbytes >> 4;
  const u32x4* src = reinterpret_cast<const u32x4*>(g);
  const Window<u32x4> w = window(src, 0, nchunk);
  u32x4* dst = reinterpret_cast<u32x4*>(lds);
  const int step = static_cast<int>(blockDim.x);
  for (int c0 = threadIdx.x; c0 < nchunk; c0 += kStageLoads * step) {
    u32x4 v[kStageLoads];
#pragma unroll
    for (int j = 0; j < kStageLoads; ++j)
      if (c0 + j * step < nchunk) v[j] = STREAM ? win_ld1(w, c0 + j * step) : src[c0 + j * step];
#pragma unroll
    for (int j = 0; j < kStageLoads; ++j)
      if (c0 + j * step < nchunk) dst[c0 + j * step] = v[j];
  }
  for (int b = (nchunk << 4) + threadIdx.x; b < nbytes; b += blockDim.x) lds[b] = g[b];
}

template <bool STREAM>
__device__ __forceinline__ void stage_out(char* g, const char* lds, int nbytes) {
  const int nchunk = nbytes >> 4;
  const u32x4* src = reinterpret_cast<const u32x4*>(lds);
  u32x4* dst = reinterpret_cast<u32x4*>(g);
  const Window<u32x4> w = window(dst, 0, nchunk);
  for (int c = threadIdx.x; c < nchunk; c += blockDim.x) {
    if constexpr (STREAM) win_st1(w, c, src[c]);
    else dst[c] = src[c];
  }
  for (int b = (nchunk << 4) + threadIdx.x; b < nbytes; b += blockDim.x) g[b] = lds[b];
}

// ------------------------------------------------------------- AoS steps

template <int INTEG, typename PT, typename VT, bool ALIGNED, int TIER, bool STREAM>
__global__ __launch_bounds__(1024) void aos_step_kernel(AosStepArgs a, int tile) {
  extern __shared__ uint4 lds_u4[];
  char* lds = reinterpret_cast<char*>(lds_u4);
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * tile;
  const int nrec = static_cast<int>(min(static_cast<int64_t>(tile), a.n - r0));
  char* g = a.aos + r0 * a.stride;
  const int nbytes = nrec * a.stride;
  stage_in<STREAM>(lds, g, nbytes);
  __syncthreads();
  const Abc p = to_abc(a.abc);
  for (int r = threadIdx.x; r < nrec; r += blockDim.x)
    update_record<INTEG, PT, VT, ALIGNED, TIER>(lds + r * a.stride, a, p);
  __syncthreads();
  stage_out<STREAM>(g, lds, nbytes);
}

template <int INTEG, typename PT, typename VT, bool ALIGNED, int TIER>
__global__ __launch_bounds__(1024) void aos_naive_kernel(AosStepArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  update_record<INTEG, PT, VT, ALIGNED, TIER>(a.aos + i * a.stride, a, to_abc(a.abc));
}

template <int INTEG, typename PT, typename VT, int TIER>
hipError_t aos_step_launch(bool aligned, bool naive, int block, const AosStepArgs& a,
                           hipStream_t s) {
  if (naive) {
    const int64_t grid = (a.n + block - 1) / block;
    if (aligned)
      hipLaunchKernelGGL((aos_naive_kernel<INTEG, PT, VT, true, TIER>), dim3(grid), dim3(block), 0,
                         s, a);
    else
      hipLaunchKernelGGL((aos_naive_kernel<INTEG, PT, VT, false, TIER>), dim3(grid), dim3(block),
                         0, s, a);
  } else {
    const int tile = aos_tile_records(a.stride, block);
    const int64_t grid = (a.n + tile - 1) / tile;
    const size_t lds = (static_cast<size_t>(tile) * a.stride + 15) & ~static_cast<size_t>(15);
    const bool stream = a.n * a.stride >= kStreamBytes;
    if (aligned && stream)
      hipLaunchKernelGGL((aos_step_kernel<INTEG, PT, VT, true, TIER, true>), dim3(grid),
                         dim3(block), lds, s, a, tile);
    else if (aligned)
      hipLaunchKernelGGL((aos_step_kernel<INTEG, PT, VT, true, TIER, false>), dim3(grid),
                         dim3(block), lds, s, a, tile);
    else if (stream)
      hipLaunchKernelGGL((aos_step_kernel<INTEG, PT, VT, false, TIER, true>), dim3(grid),
                         dim3(block), lds, s, a, tile);
    else
      hipLaunchKernelGGL((aos_step_kernel<INTEG, PT, VT, false, TIER, false>), dim3(grid),
                         dim3(block), lds, s, a, tile);
  }
  return hipGetLastError();
}

template <int INTEG, typename PT, typename VT>
hipError_t aos_step_t(bool aligned, bool naive, int block, const AosStepArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if constexpr (field_integrator(INTEG)) {
    const int tier = shift_tier(a.dt, a.abc.A, a.abc.B, a.abc.C);
    if (tier == kTierSmall)
      return aos_step_launch<INTEG, PT, VT, kTierSmall>(aligned, naive, block, a, s);
    if (tier == kTierMid)
      return aos_step_launch<INTEG, PT, VT, kTierMid>(aligned, naive, block, a, s);
  }
  return aos_step_launch<INTEG, PT, VT, kTierAny>(aligned, naive, block, a, s);
}

template <int INTEG>
hipError_t aos_dispatch(int pos_t, int vel_t, bool aligned, bool naive, int block,
                        const AosStepArgs& a, hipStream_t s) {
  if (pos_t == kF64 && vel_t == kF32) return aos_step_t<INTEG, double, float>(aligned, naive, block, a, s);
  if (pos_t == kF64 && vel_t == kF64) return aos_step_t<INTEG, double, double>(aligned, naive, block, a, s);
  if constexpr (!field_integrator(INTEG)) {
    if (pos_t == kF32 && vel_t == kF32) return aos_step_t<INTEG, float, float>(aligned, naive, block, a, s);
    if (pos_t == kF32 && vel_t == kF64) return aos_step_t<INTEG, float, double>(aligned, naive, block, a, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------- transposes

// Arrays whose elements one thread loads before it stores any of them, so
// that a wave has several independent loads in flight.  The arrays come in
// groups of one element size (XposeArgs::order); each group is walked in
// blocks of kXposeGroup arrays and one final block of the remainder, every
// block straight-line code: all its loads, then all its stores.
constexpr int kXposeGroup = 4;

template <typename F>
__device__ __forceinline__ void for_blocks(int b, int e, F&& f) {
  int a0 = b;
  for (; a0 + kXposeGroup <= e; a0 += kXposeGroup) f(std::integral_constant<int, kXposeGroup>{}, a0);
  switch (e - a0) {
    case 3: f(std::integral_constant<int, 3>{}, a0); break;
    case 2: f(std::integral_constant<int, 2>{}, a0); break;
    case 1: f(std::integral_constant<int, 1>{}, a0); break;
    default: break;
  }
}

// Element r0 + r of arrays order[b..e) (element type T) into the record
// `rec`.  STREAM: through buffer windows over the tile's nrec elements of
// each array, with the streaming cache policies.
template <typename T, bool ALIGNED, bool STREAM>
__device__ __forceinline__ void gather_size(const XposeArgs& t, int b, int e, int64_t r0,
                                            int nrec, int r, char* rec) {
  for_blocks(b, e, [&](auto G, int a0) {
    T v[G.value];
#pragma unroll
    for (int j = 0; j < G.value; ++j) {
      const T* arr = reinterpret_cast<const T*>(t.soa[t.order[a0 + j]]);
      if constexpr (STREAM) v[j] = win_ld1(window(arr, r0, nrec), r);
      else v[j] = arr[r0 + r];
    }
#pragma unroll
    for (int j = 0; j < G.value; ++j) rec_store<T, ALIGNED>(rec + t.off[t.order[a0 + j]], v[j]);
  });
}

// The record `rec`'s fields of arrays order[b..e) into element r0 + r of
// each (STREAM as in gather_size).
template <typename T, bool ALIGNED, bool STREAM>
__device__ __forceinline__ void scatter_size(const XposeArgs& t, int b, int e, int64_t r0,
                                             int nrec, int r, const char* rec) {
  for_blocks(b, e, [&](auto G, int a0) {
    T v[G.value];
#pragma unroll
    for (int j = 0; j < G.value; ++j) v[j] = rec_load<T, ALIGNED>(rec + t.off[t.order[a0 + j]]);
#pragma unroll
    for (int j = 0; j < G.value; ++j) {
      T* arr = reinterpret_cast<T*>(t.soa[t.order[a0 + j]]);
      if constexpr (STREAM) win_st1(window(arr, r0, nrec), r, v[j]);
      else arr[r0 + r] = v[j];
    }
  });
}

// AoS -> SoA: the tile's records are staged through LDS with coalesced 16-byte
// loads; then thread r moves every field of record r from LDS to element r of
// its array, a block of arrays of one element size at a time (uniform across
// the workgroup), so consecutive lanes store consecutive elements.
template <bool ALIGNED, bool STREAM>
__global__ __launch_bounds__(256) void aos_to_soa_kernel(const XposeArgs* __restrict__ tp,
                                                         int64_t n, int tile) {
  extern __shared__ uint4 lds_u4[];
  char* lds = reinterpret_cast<char*>(lds_u4);
  const XposeArgs& t = *tp;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * tile;
  const int nrec = static_cast<int>(min(static_cast<int64_t>(tile), n - r0));
  const int stride = t.stride;
  stage_in<STREAM>(lds, t.aos + r0 * stride, nrec * stride);
  __syncthreads();
  for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
    const char* rec = lds + r * stride;
    scatter_size<uint64_t, ALIGNED, STREAM>(t, 0, t.group_end[0], r0, nrec, r, rec);
    scatter_size<uint32_t, ALIGNED, STREAM>(t, t.group_end[0], t.group_end[1], r0, nrec, r, rec);
    scatter_size<uint8_t, ALIGNED, false>(t, t.group_end[1], t.group_end[2], r0, nrec, r, rec);
  }
}

// SoA -> AoS: zero the LDS tile (padding bytes are whatever no field writes),
// gather element r of every array into record r, a block of arrays of one
// element size at a time, then store the tile with coalesced 16-byte stores.
template <bool ALIGNED, bool STREAM>
__global__ __launch_bounds__(256) void soa_to_aos_kernel(const XposeArgs* __restrict__ tp,
                                                         int64_t n, int tile) {
  extern __shared__ uint4 lds_u4[];
  char* lds = reinterpret_cast<char*>(lds_u4);
  const XposeArgs& t = *tp;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * tile;
  const int nrec = static_cast<int>(min(static_cast<int64_t>(tile), n - r0));
  const int stride = t.stride;
  const int nbytes = nrec * stride;
  for (int c = threadIdx.x; c < (nbytes + 15) >> 4; c += blockDim.x)
    lds_u4[c] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
    char* rec = lds + r * stride;
    gather_size<uint64_t, ALIGNED, STREAM>(t, 0, t.group_end[0], r0, nrec, r, rec);
    gather_size<uint32_t, ALIGNED, STREAM>(t, t.group_end[0], t.group_end[1], r0, nrec, r, rec);
    gather_size<uint8_t, ALIGNED, false>(t, t.group_end[1], t.group_end[2], r0, nrec, r, rec);
  }
  __syncthreads();
  stage_out<STREAM>(t.aos + r0 * stride, lds, nbytes);
}

// ------------------------------------------------------------ AoSoA tiles


// SoA <-> AoSoA for arrays order[b..e) (element type T): lane `lane` of
// `tile` is particle i.  Lanes past n (the last tile's padding) are written
// as zero bytes on the tile side and never stored on the SoA side; they load
// element n - 1 (n >= 1) so that no load needs a branch.
template <typename T, bool TO_SOA>
__device__ __forceinline__ void aosoa_size(const XposeArgs& t, int b, int e, char* tile, int lane,
                                           int64_t i, int64_t n) {
  const bool live = i < n;
  const int64_t ic = live ? i : n - 1;
  for_blocks(b, e, [&](auto G, int a0) {
    T v[G.value];
#pragma unroll
    for (int j = 0; j < G.value; ++j) {
      const int a = t.order[a0 + j];
      if constexpr (TO_SOA) {
        v[j] = reinterpret_cast<const T*>(tile + t.off[a])[lane];
      } else {
        const T x = reinterpret_cast<const T*>(t.soa[a])[ic];
        v[j] = live ? x : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < G.value; ++j) {
      const int a = t.order[a0 + j];
      if constexpr (TO_SOA) {
        if (live) reinterpret_cast<T*>(t.soa[a])[i] = v[j];
      } else {
        reinterpret_cast<T*>(tile + t.off[a])[lane] = v[j];
      }
    }
  });
}

// SoA <-> AoSoA: one thread per particle lane from lane `first` on; the 64
// lanes of a wave cover one tile, so both sides of every copy are contiguous
// runs.  Used for the last, partial tile, and for every tile when an array
// is not 16-byte aligned.
template <bool TO_SOA>
__global__ __launch_bounds__(256) void aosoa_xpose_kernel(const XposeArgs* __restrict__ tp,
                                                          int64_t n, int64_t first) {
  const XposeArgs& t = *tp;
  const int64_t i = first + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t lanes = (n + kAosoaW - 1) / kAosoaW * kAosoaW;
  if (i >= lanes) return;
  char* tile = t.aos + (i / kAosoaW) * t.stride;
  const int lane = static_cast<int>(i % kAosoaW);
  aosoa_size<uint64_t, TO_SOA>(t, 0, t.group_end[0], tile, lane, i, n);
  aosoa_size<uint32_t, TO_SOA>(t, t.group_end[0], t.group_end[1], tile, lane, i, n);
  aosoa_size<uint8_t, TO_SOA>(t, t.group_end[1], t.group_end[2], tile, lane, i, n);
}

// SoA <-> AoSoA for the `full` whole tiles: each array's 64 elements form
// one 16-byte aligned run on both sides (a tile holds no padding and every
// array starts at a multiple of 64 bytes), so thread g copies 16-byte chunk
// g % chunks of tile g / chunks.  Needs 16-byte aligned SoA arrays.
template <bool TO_SOA>
__global__ __launch_bounds__(256) void aosoa_chunk_kernel(const XposeArgs* __restrict__ tp,
                                                          int64_t full, int32_t chunks) {
  const XposeArgs& t = *tp;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= full * chunks) return;
  const int64_t tile = g / chunks;
  const int32_t byte = static_cast<int32_t>(g - tile * chunks) * 16;
  int a = 0;  // the array whose run holds this chunk (offsets ascend)
  for (int k = 1; k < t.narrays; ++k)
    if (t.off[k] <= byte) a = k;
  const int64_t run = static_cast<int64_t>(kAosoaW) * t.es[a];
  u32x4* tile_p = reinterpret_cast<u32x4*>(t.aos + tile * t.stride + byte);
  u32x4* soa_p = reinterpret_cast<u32x4*>(t.soa[a] + tile * run + (byte - t.off[a]));
  if constexpr (TO_SOA) *soa_p = *tile_p;
  else *tile_p = *soa_p;
}

// Element `lane` of the tile array at byte `off` of tile base `tb`.  STREAM:
// through a buffer window over the tile's 64 elements with the streaming
// cache policies; otherwise a plain global access.
template <bool STREAM, typename T>
__device__ __forceinline__ T tile_ld(char* tb, int32_t off, int lane) {
  const T* arr = reinterpret_cast<const T*>(tb + off);
  if constexpr (STREAM) return win_ld1(window(arr, 0, kAosoaW), lane);
  else return arr[lane];
}

template <bool STREAM, typename T>
__device__ __forceinline__ void tile_st(char* tb, int32_t off, int lane, T v) {
  T* arr = reinterpret_cast<T*>(tb + off);
  if constexpr (STREAM) win_st1(window(arr, 0, kAosoaW), lane, v);
  else arr[lane] = v;
}

template <int INTEG, typename PT, typename VT, int TIER, bool STREAM>
__global__ __launch_bounds__(1024) void aosoa_step_kernel(AosoaStepArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Abc p = to_abc(a.abc);
  // a workgroup is whole waves (the host launches multiples of 64 threads)
  // and a tile is 64 particles, so every lane of a wave is in the same tile
  const int64_t tile = __builtin_amdgcn_readfirstlane(static_cast<int>(i / kAosoaW));
  const int lane = static_cast<int>(i - tile * kAosoaW);
  char* tb = a.base + tile * a.tile_bytes;
  if constexpr (!field_integrator(INTEG) && STREAM) {
    // one component at a time, as in the streaming SoA kernel
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      PT x = tile_ld<true, PT>(tb, a.off_pos[d], lane);
      VT v = tile_ld<true, VT>(tb, a.off_vel[d], lane);
      const VT g = uses_acc(INTEG) ? tile_ld<true, VT>(tb, a.off_acc[d], lane) : VT(0);
      euler_component<INTEG, PT, VT>(x, v, g, a.dt, a.wrap);
      tile_st<true>(tb, a.off_pos[d], lane, x);
      if constexpr (uses_acc(INTEG)) tile_st<true>(tb, a.off_vel[d], lane, v);
    }
  } else {
    // every load before the first store (cache-resident sets are bound by
    // latency; see the SoA kernel)
    PT x = tile_ld<STREAM, PT>(tb, a.off_pos[0], lane), y = tile_ld<STREAM, PT>(tb, a.off_pos[1], lane),
       z = tile_ld<STREAM, PT>(tb, a.off_pos[2], lane);
    VT u = VT(0), v = VT(0), w = VT(0), g0 = VT(0), g1 = VT(0), g2 = VT(0);
    if constexpr (!field_integrator(INTEG)) {
      u = tile_ld<STREAM, VT>(tb, a.off_vel[0], lane);
      v = tile_ld<STREAM, VT>(tb, a.off_vel[1], lane);
      w = tile_ld<STREAM, VT>(tb, a.off_vel[2], lane);
    }
    if constexpr (uses_acc(INTEG)) {
      g0 = tile_ld<STREAM, VT>(tb, a.off_acc[0], lane);
      g1 = tile_ld<STREAM, VT>(tb, a.off_acc[1], lane);
      g2 = tile_ld<STREAM, VT>(tb, a.off_acc[2], lane);
    }
    update_particle<INTEG, PT, VT, TIER>(x, y, z, u, v, w, g0, g1, g2, a.dt, p, a.wrap);
    tile_st<STREAM>(tb, a.off_pos[0], lane, x);
    tile_st<STREAM>(tb, a.off_pos[1], lane, y);
    tile_st<STREAM>(tb, a.off_pos[2], lane, z);
    if constexpr (INTEG != kEuler) {
      tile_st<STREAM>(tb, a.off_vel[0], lane, u);
      tile_st<STREAM>(tb, a.off_vel[1], lane, v);
      tile_st<STREAM>(tb, a.off_vel[2], lane, w);
    }
  }
}

template <int INTEG, typename PT, typename VT>
hipError_t aosoa_step_t(int block, const AosoaStepArgs& a, hipStream_t s) {
  const int64_t grid = (a.n + block - 1) / block;
  int64_t bytes = 3 * (sizeof(PT) + sizeof(VT));
  if (uses_acc(INTEG)) bytes += 3 * sizeof(VT);
  const bool stream = a.n * bytes >= kStreamBytes;
  int tier = kTierAny;
  if constexpr (field_integrator(INTEG)) tier = shift_tier(a.dt, a.abc.A, a.abc.B, a.abc.C);
#define SOAX_AOSOA(TI, ST) \
  hipLaunchKernelGGL((aosoa_step_kernel<INTEG, PT, VT, TI, ST>), dim3(grid), dim3(block), 0, s, a)
  if (tier == kTierSmall && stream) SOAX_AOSOA(kTierSmall, true);
  else if (tier == kTierSmall) SOAX_AOSOA(kTierSmall, false);
  else if (tier == kTierMid && stream) SOAX_AOSOA(kTierMid, true);
  else if (tier == kTierMid) SOAX_AOSOA(kTierMid, false);
  else if (stream) SOAX_AOSOA(kTierAny, true);
  else SOAX_AOSOA(kTierAny, false);
#undef SOAX_AOSOA
  return hipGetLastError();
}

template <int INTEG>
hipError_t aosoa_dispatch(int pos_t, int vel_t, int block, const AosoaStepArgs& a, hipStream_t s) {
  if (pos_t == kF64 && vel_t == kF32) return aosoa_step_t<INTEG, double, float>(block, a, s);
  if (pos_t == kF64 && vel_t == kF64) return aosoa_step_t<INTEG, double, double>(block, a, s);
  if constexpr (!field_integrator(INTEG)) {
    if (pos_t == kF32 && vel_t == kF32) return aosoa_step_t<INTEG, float, float>(block, a, s);
    if (pos_t == kF32 && vel_t == kF64) return aosoa_step_t<INTEG, float, double>(block, a, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------- fill

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// i-th output of a SplitMix64 generator seeded with the s-th output of one
// seeded with `seed`.
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t s, uint64_t i) {
  return mix64(mix64(seed + kGamma * (s + 1)) + kGamma * (i + 1));
}

__device__ __forceinline__ double unit_co(uint64_t r) {  // [0, 1)
  return static_cast<double>(r >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ double unit_oc(uint64_t r) {  // (0, 1]
  return static_cast<double>((r >> 11) + 1) * 0x1.0p-53;
}

__device__ __forceinline__ void store_value(void* arr, int64_t i, int dtype, double f, uint64_t bits,
                                            bool is_real) {
  switch (dtype) {
    case kF64: static_cast<double*>(arr)[i] = is_real ? f : static_cast<double>(bits); break;
    case kF32: static_cast<float*>(arr)[i] = static_cast<float>(is_real ? f : static_cast<double>(bits)); break;
    case kI64: static_cast<uint64_t*>(arr)[i] = bits; break;
    case kI32: static_cast<uint32_t*>(arr)[i] = static_cast<uint32_t>(bits); break;
    default: static_cast<uint8_t*>(arr)[i] = static_cast<uint8_t>(bits); break;
  }
}

__global__ __launch_bounds__(256) void fill_kernel(FillArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t r = draw(a.seed, a.stream, static_cast<uint64_t>(i));
  switch (a.rule) {
    case kFillIndex: store_value(a.arr, i, a.dtype, 0.0, static_cast<uint64_t>(i), false); break;
    case kFillRaw: store_value(a.arr, i, a.dtype, 0.0, r, false); break;
    case kFillTop8: store_value(a.arr, i, a.dtype, 0.0, r >> 56, false); break;
    case kFillBox: store_value(a.arr, i, a.dtype, kBoxL * unit_co(r), 0, true); break;
    case kFillMass: store_value(a.arr, i, a.dtype, 0.5 + 1.5 * unit_co(r), 0, true); break;
    case kFillUnit: store_value(a.arr, i, a.dtype, unit_co(r), 0, true); break;
    default: {  // Box-Muller
      const double u1 = unit_oc(r);
      const double u2 = unit_co(draw(a.seed, a.stream + 1, static_cast<uint64_t>(i)));
      store_value(a.arr, i, a.dtype, sqrt(-2.0 * log(u1)) * cos(kBoxL * u2), 0, true);
      break;
    }
  }
}

template <typename PT, typename VT>
__global__ __launch_bounds__(256) void vel_from_field_kernel(SoaStepArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const PT* px = static_cast<const PT*>(a.pos[0]);
  const PT* py = static_cast<const PT*>(a.pos[1]);
  const PT* pz = static_cast<const PT*>(a.pos[2]);
  double u0, u1, u2;
  abc_field(to_abc(a.abc), widen(px[i]), widen(py[i]), widen(pz[i]), u0, u1, u2);
  static_cast<VT*>(a.vel[0])[i] = static_cast<VT>(u0);
  static_cast<VT*>(a.vel[1])[i] = static_cast<VT>(u1);
  static_cast<VT*>(a.vel[2])[i] = static_cast<VT>(u2);
}

// ------------------------------------------------------------------- copy

// One 16-byte element per thread, moved through buffer windows over the
// workgroup's run with the streaming cache policies of the step kernels: the
// fastest streaming form measured on the MI355X (a grid-stride loop or
// several elements per thread keep fewer independent requests in flight per
// CU).

__global__ __launch_bounds__(256) void copy16_kernel(u32x4* __restrict__ dst,
                                                     const u32x4* __restrict__ src, int64_t n16) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n16) return;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x;
  const int64_t cnt = min(static_cast<int64_t>(blockDim.x), n16 - first);
  const int e = static_cast<int>(threadIdx.x);
  win_st1(window(dst, first, cnt), e, win_ld1(window(src, first, cnt), e));
}

__global__ void copy_tail_kernel(char* dst, const char* src, int64_t from, int64_t bytes) {
  const int64_t i = from + threadIdx.x;
  if (i < bytes) dst[i] = src[i];
}

// ------------------------------------------------------------ stream probes

// The memory accesses of the streaming SoA step kernels with their
// arithmetic taken out: one particle per thread, every load and store through
// the same buffer windows and cache-policy bits as
// soa_step_kernel<..., STREAM = true>.  a.c is 0 for the patterns that write
// (positions are rewritten unchanged) and NaN for the read-only one, whose
// single guarded store never fires but keeps the loads alive.
template <int PAT>
__global__ __launch_bounds__(1024) void stream_probe_kernel(ProbeArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x;
  const int64_t cnt = min(static_cast<int64_t>(blockDim.x), a.n - first);
  const int e = static_cast<int>(threadIdx.x);
  Window<double> P[3];
  Window<float> V[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    P[d] = window(a.pos[d], first, cnt);
    V[d] = window(a.vel[d], first, cnt);
  }
  if constexpr (PAT == kProbeRk2) {
    const double x = win_ld1(P[0], e), y = win_ld1(P[1], e), z = win_ld1(P[2], e);
    win_st1(P[0], e, x + a.c);
    win_st1(P[1], e, y + a.c);
    win_st1(P[2], e, z + a.c);
    win_st1(V[0], e, static_cast<float>(x));
    win_st1(V[1], e, static_cast<float>(y));
    win_st1(V[2], e, static_cast<float>(z));
  } else if constexpr (PAT == kProbeEuler) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = win_ld1(P[d], e);
      const float v = win_ld1(V[d], e);
      win_st1(P[d], e, x + a.c * static_cast<double>(v));
    }
  } else if constexpr (PAT == kProbeRead) {
    const double s = (win_ld1(P[0], e) + win_ld1(P[1], e)) + win_ld1(P[2], e);
    if (s == a.c) a.pos[0][i] = s;
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      win_st1(P[d], e, a.c);
      win_st1(V[d], e, static_cast<float>(a.c));
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_soa_fused(int integ, int pos_t, int vel_t, int block, const SoaStepArgs& a,
                            int64_t nsteps, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const bool pd = pos_t == kF64, vd = vel_t == kF64;
  switch (integ) {
    case kEuler:
      if (pd && !vd) return soa_fused_launch<kEuler, double, float>(block, a, nsteps, s);
      if (pd && vd) return soa_fused_launch<kEuler, double, double>(block, a, nsteps, s);
      if (!pd && !vd) return soa_fused_launch<kEuler, float, float>(block, a, nsteps, s);
      return soa_fused_launch<kEuler, float, double>(block, a, nsteps, s);
    case kEulerAcc:
      if (pd && !vd) return soa_fused_launch<kEulerAcc, double, float>(block, a, nsteps, s);
      if (pd && vd) return soa_fused_launch<kEulerAcc, double, double>(block, a, nsteps, s);
      if (!pd && !vd) return soa_fused_launch<kEulerAcc, float, float>(block, a, nsteps, s);
      return soa_fused_launch<kEulerAcc, float, double>(block, a, nsteps, s);
    case kSymEuler:
      if (pd && !vd) return soa_fused_launch<kSymEuler, double, float>(block, a, nsteps, s);
      if (pd && vd) return soa_fused_launch<kSymEuler, double, double>(block, a, nsteps, s);
      if (!pd && !vd) return soa_fused_launch<kSymEuler, float, float>(block, a, nsteps, s);
      return soa_fused_launch<kSymEuler, float, double>(block, a, nsteps, s);
    case kRk2Abc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_fused_launch<kRk2Abc, double, double>(block, a, nsteps, s);
      return soa_fused_launch<kRk2Abc, double, float>(block, a, nsteps, s);
    case kHeunAbc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_fused_launch<kHeunAbc, double, double>(block, a, nsteps, s);
      return soa_fused_launch<kHeunAbc, double, float>(block, a, nsteps, s);
    case kRk4Abc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_fused_launch<kRk4Abc, double, double>(block, a, nsteps, s);
      return soa_fused_launch<kRk4Abc, double, float>(block, a, nsteps, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_soa_step(int integ, int pos_t, int vel_t, int vec, int block,
                           const SoaStepArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const bool pd = pos_t == kF64, vd = vel_t == kF64;
  switch (integ) {
    case kEuler:
      if (pd && !vd) return soa_step_vec<kEuler, double, float>(vec, block, a, s);
      if (pd && vd) return soa_step_vec<kEuler, double, double>(vec, block, a, s);
      if (!pd && !vd) return soa_step_vec<kEuler, float, float>(vec, block, a, s);
      return soa_step_vec<kEuler, float, double>(vec, block, a, s);
    case kEulerAcc:
      if (pd && !vd) return soa_step_vec<kEulerAcc, double, float>(vec, block, a, s);
      if (pd && vd) return soa_step_vec<kEulerAcc, double, double>(vec, block, a, s);
      if (!pd && !vd) return soa_step_vec<kEulerAcc, float, float>(vec, block, a, s);
      return soa_step_vec<kEulerAcc, float, double>(vec, block, a, s);
    case kRk2Abc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_step_vec<kRk2Abc, double, double>(vec, block, a, s);
      return soa_step_vec<kRk2Abc, double, float>(vec, block, a, s);
    case kHeunAbc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_step_vec<kHeunAbc, double, double>(vec, block, a, s);
      return soa_step_vec<kHeunAbc, double, float>(vec, block, a, s);
    case kRk4Abc:
      if (!pd) return hipErrorInvalidValue;
      if (vd) return soa_step_vec<kRk4Abc, double, double>(vec, block, a, s);
      return soa_step_vec<kRk4Abc, double, float>(vec, block, a, s);
    case kSymEuler:
      if (pd && !vd) return soa_step_vec<kSymEuler, double, float>(vec, block, a, s);
      if (pd && vd) return soa_step_vec<kSymEuler, double, double>(vec, block, a, s);
      if (!pd && !vd) return soa_step_vec<kSymEuler, float, float>(vec, block, a, s);
      return soa_step_vec<kSymEuler, float, double>(vec, block, a, s);
    default:
      return hipErrorInvalidValue;
  }
}

int aos_tile_records(int stride, int block) {
  int tile = block;
  const int cap = (kLdsBudget / stride) & ~15;
  if (tile > cap) tile = cap;
  if (tile < 16) tile = 16;
  return tile;
}

static hipError_t aos_any(int integ, int pos_t, int vel_t, bool aligned, bool naive, int block,
                          const AosStepArgs& a, hipStream_t s) {
  switch (integ) {
    case kEuler: return aos_dispatch<kEuler>(pos_t, vel_t, aligned, naive, block, a, s);
    case kEulerAcc: return aos_dispatch<kEulerAcc>(pos_t, vel_t, aligned, naive, block, a, s);
    case kRk2Abc: return aos_dispatch<kRk2Abc>(pos_t, vel_t, aligned, naive, block, a, s);
    case kHeunAbc: return aos_dispatch<kHeunAbc>(pos_t, vel_t, aligned, naive, block, a, s);
    case kRk4Abc: return aos_dispatch<kRk4Abc>(pos_t, vel_t, aligned, naive, block, a, s);
    case kSymEuler: return aos_dispatch<kSymEuler>(pos_t, vel_t, aligned, naive, block, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_aos_step(int integ, int pos_t, int vel_t, bool aligned, int block,
                           const AosStepArgs& a, hipStream_t s) {
  return aos_any(integ, pos_t, vel_t, aligned, false, block, a, s);
}

hipError_t launch_aos_naive(int integ, int pos_t, int vel_t, bool aligned, int block,
                            const AosStepArgs& a, hipStream_t s) {
  return aos_any(integ, pos_t, vel_t, aligned, true, block, a, s);
}

static int xpose_tile(int stride) {
  // 256 records per tile unless the staging would exceed the LDS budget;
  // always a multiple of 16 so every tile starts on a 16-byte boundary.
  return aos_tile_records(stride, 256);
}

hipError_t launch_xpose(bool to_soa, const XposeArgs& host, const XposeArgs* dev,
                            hipStream_t s) {
  if (host.n == 0) return hipSuccess;
  const int tile = xpose_tile(host.stride);
  const int64_t grid = (host.n + tile - 1) / tile;
  const size_t lds = (static_cast<size_t>(tile) * host.stride + 15) & ~static_cast<size_t>(15);
  const bool stream = host.n * host.stride >= kStreamBytes;
#define SOAX_XPOSE(KER)                                                                       \
  if (host.aligned && stream)                                                                 \
    hipLaunchKernelGGL((KER<true, true>), dim3(grid), dim3(256), lds, s, dev, host.n, tile);  \
  else if (host.aligned)                                                                      \
    hipLaunchKernelGGL((KER<true, false>), dim3(grid), dim3(256), lds, s, dev, host.n, tile); \
  else if (stream)                                                                            \
    hipLaunchKernelGGL((KER<false, true>), dim3(grid), dim3(256), lds, s, dev, host.n, tile); \
  else                                                                                        \
    hipLaunchKernelGGL((KER<false, false>), dim3(grid), dim3(256), lds, s, dev, host.n, tile);
  if (to_soa) {
    SOAX_XPOSE(aos_to_soa_kernel)
  } else {
    SOAX_XPOSE(soa_to_aos_kernel)
  }
#undef SOAX_XPOSE
  return hipGetLastError();
}

hipError_t launch_aosoa_xpose(bool to_soa, const XposeArgs& host, const XposeArgs* dev,
                              hipStream_t s) {
  if (host.n == 0) return hipSuccess;
  const int64_t lanes = (host.n + kAosoaW - 1) / kAosoaW * kAosoaW;
  bool aligned = true;  // whole tiles go by 16-byte chunks when every array allows it
  for (int a = 0; a < host.narrays; ++a)
    if (reinterpret_cast<uintptr_t>(host.soa[a]) & 15u) aligned = false;
  int64_t first = 0;
  const int64_t full = host.n / kAosoaW;
  if (aligned && full > 0 && host.stride % 16 == 0) {
    const int32_t chunks = host.stride / 16;
    const int64_t grid = (full * chunks + 255) / 256;
    if (to_soa)
      hipLaunchKernelGGL(aosoa_chunk_kernel<true>, dim3(grid), dim3(256), 0, s, dev, full, chunks);
    else
      hipLaunchKernelGGL(aosoa_chunk_kernel<false>, dim3(grid), dim3(256), 0, s, dev, full, chunks);
    first = full * kAosoaW;
  }
  if (first < lanes) {
    const int64_t grid = (lanes - first + 255) / 256;
    if (to_soa)
      hipLaunchKernelGGL(aosoa_xpose_kernel<true>, dim3(grid), dim3(256), 0, s, dev, host.n, first);
    else
      hipLaunchKernelGGL(aosoa_xpose_kernel<false>, dim3(grid), dim3(256), 0, s, dev, host.n, first);
  }
  return hipGetLastError();
}

hipError_t launch_aosoa_step(int integ, int pos_t, int vel_t, int block, const AosoaStepArgs& a,
                             hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (integ) {
    case kEuler: return aosoa_dispatch<kEuler>(pos_t, vel_t, block, a, s);
    case kEulerAcc: return aosoa_dispatch<kEulerAcc>(pos_t, vel_t, block, a, s);
    case kRk2Abc: return aosoa_dispatch<kRk2Abc>(pos_t, vel_t, block, a, s);
    case kHeunAbc: return aosoa_dispatch<kHeunAbc>(pos_t, vel_t, block, a, s);
    case kRk4Abc: return aosoa_dispatch<kRk4Abc>(pos_t, vel_t, block, a, s);
    case kSymEuler: return aosoa_dispatch<kSymEuler>(pos_t, vel_t, block, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill(const FillArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t grid = (a.n + 255) / 256;
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vel_from_field(int pos_t, int vel_t, const SoaStepArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t grid = (a.n + 255) / 256;
  if (pos_t == kF64 && vel_t == kF32)
    hipLaunchKernelGGL((vel_from_field_kernel<double, float>), dim3(grid), dim3(256), 0, s, a);
  else if (pos_t == kF64 && vel_t == kF64)
    hipLaunchKernelGGL((vel_from_field_kernel<double, double>), dim3(grid), dim3(256), 0, s, a);
  else if (pos_t == kF32 && vel_t == kF32)
    hipLaunchKernelGGL((vel_from_field_kernel<float, float>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((vel_from_field_kernel<float, double>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, int64_t bytes, hipStream_t s) {
  const int64_t n16 = bytes >> 4;
  if (n16 > 0) {
    const int64_t grid = (n16 + 255) / 256;
    hipLaunchKernelGGL(copy16_kernel, dim3(grid), dim3(256), 0, s, static_cast<u32x4*>(dst),
                       static_cast<const u32x4*>(src), n16);
  }
  if (bytes & 15) {
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(16), 0, s, static_cast<char*>(dst),
                       static_cast<const char*>(src), n16 << 4, bytes);
  }
  return hipGetLastError();
}

hipError_t launch_stream_probe(int pattern, const ProbeArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int block = 128;  // the SoA step's default workgroup
  const int64_t grid = (a.n + block - 1) / block;
  switch (pattern) {
    case kProbeRk2:
      hipLaunchKernelGGL(stream_probe_kernel<kProbeRk2>, dim3(grid), dim3(block), 0, s, a);
      break;
    case kProbeEuler:
      hipLaunchKernelGGL(stream_probe_kernel<kProbeEuler>, dim3(grid), dim3(block), 0, s, a);
      break;
    case kProbeRead:
      hipLaunchKernelGGL(stream_probe_kernel<kProbeRead>, dim3(grid), dim3(block), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL(stream_probe_kernel<kProbeWrite>, dim3(grid), dim3(block), 0, s, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace soax
