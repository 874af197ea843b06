// k_batch.hip -- one persistent launch advancing many particle sets of
// uneven sizes by one RK2 step each, every set with its own dt and field
// amplitudes.
//
// The sets are cut into tiles of `tile` particles (the last tile of a set may
// be short) and listed back to back; each workgroup reads its tile's set from
// a device table.  Either every tile has a workgroup of its own, or a grid of
// a few workgroups per compute unit walks the list with a grid stride.  Small
// sets therefore share the machine instead of each paying for a launch of its
// own.  The per-particle arithmetic is the same
// inline function the single-set kernels use, so a set advanced here is
// bit-identical to the same set advanced alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "launch.h"

namespace soax {

namespace {

// One tile of set S.  TIER: shift_tier of this set.
template <typename VT, int PPT, int TIER>
__device__ __forceinline__ void batch_tile(const BatchSet& S, int64_t t, int32_t tile) {
  const Abc p{S.A, S.B, S.C};
  const double dt = S.dt;
  const int64_t i0 = (t - S.tile_begin) * tile + static_cast<int64_t>(threadIdx.x) * PPT;
  double* px = S.pos[0];
  double* py = S.pos[1];
  double* pz = S.pos[2];
  VT* vx = static_cast<VT*>(S.vel[0]);
  VT* vy = static_cast<VT*>(S.vel[1]);
  VT* vz = static_cast<VT*>(S.vel[2]);
  if (i0 + PPT <= S.n) {
    // the batch spans far more than the caches: streaming loads and stores
    // through buffer windows over this tile
    const int64_t first = (t - S.tile_begin) * tile;
    const int64_t cnt = min(static_cast<int64_t>(tile), S.n - first);
    const int e = static_cast<int>(threadIdx.x) * PPT;
    double x[PPT], y[PPT], z[PPT];
    VT u[PPT], v[PPT], w[PPT];
    win_ld_run<double, PPT>(window(px, first, cnt), e, x);
    win_ld_run<double, PPT>(window(py, first, cnt), e, y);
    win_ld_run<double, PPT>(window(pz, first, cnt), e, z);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      u[j] = v[j] = w[j] = VT(0);
      update_particle<kRk2Abc, double, VT, TIER>(x[j], y[j], z[j], u[j], v[j], w[j], VT(0),
                                                  VT(0), VT(0), dt, p, 1);
    }
    win_st_run<double, PPT>(window(px, first, cnt), e, x);
    win_st_run<double, PPT>(window(py, first, cnt), e, y);
    win_st_run<double, PPT>(window(pz, first, cnt), e, z);
    win_st_run<VT, PPT>(window(vx, first, cnt), e, u);
    win_st_run<VT, PPT>(window(vy, first, cnt), e, v);
    win_st_run<VT, PPT>(window(vz, first, cnt), e, w);
  } else {
    for (int64_t i = i0; i < S.n; ++i) {
      double x = px[i], y = py[i], z = pz[i];
      VT u = VT(0), v = VT(0), w = VT(0);
      update_particle<kRk2Abc, double, VT, TIER>(x, y, z, u, v, w, VT(0), VT(0), VT(0), dt, p,
                                                  1);
      px[i] = x;
      py[i] = y;
      pz[i] = z;
      vx[i] = u;
      vy[i] = v;
      vz[i] = w;
    }
  }
}

// Every tile takes the angle-shift path of its own set's tier (a branch
// uniform over the workgroup, which works on one tile at a time).  MAXT, the
// largest tier of any set in the batch, leaves the paths of larger tiers out
// of the kernel: the unbounded tier's full-reduction fallback alone raises
// the kernel's registers (at two particles per thread from about 72 to 100
// VGPRs, seven resident waves per SIMD to four).
template <typename VT, int PPT, int MAXT>
__device__ __forceinline__ void batch_tile_any(const BatchSet& S, int64_t t, int32_t tile) {
  if (MAXT == kTierSmall || S.tier == kTierSmall)
    batch_tile<VT, PPT, kTierSmall>(S, t, tile);
  else if (MAXT == kTierMid || S.tier == kTierMid)
    batch_tile<VT, PPT, kTierMid>(S, t, tile);
  else
    batch_tile<VT, PPT, kTierAny>(S, t, tile);
}

template <typename VT, int PPT, int MAXT>
__global__ __launch_bounds__(512) void batch_rk2_kernel(BatchLaunch b) {
  for (int64_t t = blockIdx.x; t < b.ntiles; t += gridDim.x)
    batch_tile_any<VT, PPT, MAXT>(b.sets[b.tile_set[t]], t, b.tile);
}

// The same with one workgroup per tile (the grid covers the tile list).
// Without the grid-stride loop the kernel needs fewer registers (64 rather
// than 80 at one particle per thread), so more waves stay resident.
template <typename VT, int PPT, int MAXT>
__global__ __launch_bounds__(512) void batch_rk2_tile_kernel(BatchLaunch b) {
  const int64_t t = blockIdx.x;
  if (t >= b.ntiles) return;
  batch_tile_any<VT, PPT, MAXT>(b.sets[b.tile_set[t]], t, b.tile);
}

template <typename VT, int PPT, int MAXT>
void batch_launch_ppt(const BatchLaunch& b, hipStream_t s) {
  if (b.grid >= b.ntiles)
    hipLaunchKernelGGL((batch_rk2_tile_kernel<VT, PPT, MAXT>), dim3(b.ntiles), dim3(b.block), 0,
                       s, b);
  else
    hipLaunchKernelGGL((batch_rk2_kernel<VT, PPT, MAXT>), dim3(b.grid), dim3(b.block), 0, s, b);
}

template <typename VT, int MAXT>
void batch_launch_tier(const BatchLaunch& b, hipStream_t s) {
  switch (b.per_thread) {
    case 1: batch_launch_ppt<VT, 1, MAXT>(b, s); break;
    case 2: batch_launch_ppt<VT, 2, MAXT>(b, s); break;
    default: batch_launch_ppt<VT, 4, MAXT>(b, s); break;
  }
}

template <typename VT>
hipError_t batch_t(const BatchLaunch& b, hipStream_t s) {
  if (b.max_tier == kTierSmall)
    batch_launch_tier<VT, kTierSmall>(b, s);
  else if (b.max_tier == kTierMid)
    batch_launch_tier<VT, kTierMid>(b, s);
  else
    batch_launch_tier<VT, kTierAny>(b, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_rk2(const BatchLaunch& b, hipStream_t s) {
  if (b.ntiles == 0) return hipSuccess;
  return b.vel_t == kF64 ? batch_t<double>(b, s) : batch_t<float>(b, s);
}

}  // namespace soax
