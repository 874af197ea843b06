// k_container.hip -- gfx950 kernels for the container operations of a
// particle set: removal by overwriting with the last particle (Section 2),
// and the zero fill used when a set grows.
//
// Removal is the sequential algorithm "while particle i is flagged, copy the
// last particle over it and shrink the set", computed in parallel from its
// closed form: with m flagged particles and n' = n - m survivors, the flagged
// slots below n' (ascending) receive the unflagged particles at or above n'
// taken from the end (descending).  Three passes: per-tile flag counts (the
// host turns them into tile offsets), per-element ranks into two lists
// (holes and movers), and the moves themselves, array by array.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "launch.h"

namespace soax {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;  // elements per thread per tile
constexpr int64_t kTile = int64_t(kBlock) * kItems;

// Bit j (0..3) set iff byte j of w is nonzero: adding 0x7F to the low seven
// bits of a byte carries into its bit 7 iff they are not all zero, and no
// carry leaves the byte.
__device__ __forceinline__ uint32_t nonzero_bytes4(uint32_t w) {
  const uint32_t hi = (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
  return ((hi >> 7) & 1u) | ((hi >> 14) & 2u) | ((hi >> 21) & 4u) | ((hi >> 28) & 8u);
}

// Bit j set iff element base + j (j < kItems) is in range and flagged.  A
// whole in-range run of 16-byte aligned flags is one 16-byte load; the last
// run of the array, or unaligned flags, go byte by byte so nothing past n is
// read.
__device__ __forceinline__ uint32_t flag_bits(const uint8_t* __restrict__ flags, int64_t base,
                                              int64_t n, bool vec) {
  static_assert(kItems == 16, "one 16-byte load per thread");
  if (vec && base + kItems <= n) {
    const uint4 w = *reinterpret_cast<const uint4*>(flags + base);
    return nonzero_bytes4(w.x) | (nonzero_bytes4(w.y) << 4) | (nonzero_bytes4(w.z) << 8) |
           (nonzero_bytes4(w.w) << 12);
  }
  uint32_t f = 0;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j;
    if (i < n && flags[i]) f |= 1u << j;
  }
  return f;
}

// Inclusive scan of v over one 64-lane wave.
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v) {
  const int lane = static_cast<int>(threadIdx.x) & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive scan of v over the workgroup; returns this thread's prefix and
// writes the total to *total.  Wave scans, then the wave totals through LDS.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* total) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int32_t wave_sum[kWaves];
  const int wid = static_cast<int>(threadIdx.x) >> 6;
  const int32_t incl = wave_inclusive_scan(v);
  if ((threadIdx.x & 63) == 63) wave_sum[wid] = incl;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const int32_t t = wave_sum[w];
    before += w < wid ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();  // wave_sum may be reused by the caller's next scan
  return before + incl - v;
}

__global__ __launch_bounds__(kBlock) void count_flags_kernel(const uint8_t* __restrict__ flags,
                                                             int64_t n, int vec,
                                                             int32_t* __restrict__ counts) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile + threadIdx.x * kItems;
  int32_t total;
  block_exclusive_scan(__popc(flag_bits(flags, base, n, vec)), &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// holes_before[b]: flagged slots in tiles before b; movers_after[b]:
// unflagged particles in tiles after b -- both from the host's scan of the
// counts.  Each thread walks its kItems elements in order; one workgroup
// scan of the flagged counts gives both ranks inside the tile, because every
// thread before this one holds kItems in-range elements or the tile's last.
__global__ __launch_bounds__(kBlock) void rank_kernel(const uint8_t* __restrict__ flags, int64_t n,
                                                      int vec, int64_t n_new,
                                                      const int64_t* __restrict__ holes_before,
                                                      const int64_t* __restrict__ movers_after,
                                                      int64_t* __restrict__ hole_at,
                                                      int64_t* __restrict__ mover_at,
                                                      int64_t* __restrict__ nmoves) {
  const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kTile;
  const int64_t base = tile0 + threadIdx.x * kItems;
  const uint32_t f = flag_bits(flags, base, n, vec);
  int32_t tot_f;
  const int32_t pre_f = block_exclusive_scan(__popc(f), &tot_f);
  const int64_t in_tile = min(kTile, n - tile0);
  const int32_t in_before = static_cast<int32_t>(min(static_cast<int64_t>(threadIdx.x) * kItems, in_tile));
  const int32_t pre_u = in_before - pre_f;  // unflagged elements before this thread's
  const int32_t tot_u = static_cast<int32_t>(in_tile) - tot_f;
  int64_t hole = holes_before[blockIdx.x] + pre_f;  // flagged slots before element i
  int32_t upto_u = pre_u;                           // unflagged in the tile up to element i
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + j;
    if (i >= n) break;
    if (f & (1u << j)) {
      if (i < n_new) hole_at[hole] = i;
      ++hole;
    } else {
      ++upto_u;
      if (i >= n_new) mover_at[movers_after[blockIdx.x] + (tot_u - upto_u)] = i;
    }
    // the flagged slots below n_new are the first `hole` ones once i = n_new - 1
    if (i == n_new - 1) *nmoves = hole;
  }
}

struct alignas(16) Word16 {
  uint32_t v[4];
};

template <int W>
struct WordOf;
template <>
struct WordOf<1> {
  using T = uint8_t;
};
template <>
struct WordOf<4> {
  using T = uint32_t;
};
template <>
struct WordOf<8> {
  using T = uint64_t;
};
template <>
struct WordOf<16> {
  using T = Word16;
};

// Grid (moves, arrays): thread x of row y moves words of element
// hole_at[k] <- mover_at[k] of array y.  Holes lie below the new size and
// movers at or above it, so no thread reads what another writes.
template <int W>
__device__ __forceinline__ void move_words(char* base, int64_t stride, int64_t h, int64_t m) {
  using T = typename WordOf<W>::T;
  T* dst = reinterpret_cast<T*>(base + h * stride);
  const T* src = reinterpret_cast<const T*>(base + m * stride);
  const int words = static_cast<int>(stride / W);
  for (int w = 0; w < words; ++w) dst[w] = src[w];
}

__global__ __launch_bounds__(kBlock) void move_all_kernel(MoveArgs a,
                                                          const int64_t* __restrict__ hole_at,
                                                          const int64_t* __restrict__ mover_at,
                                                          const int64_t* __restrict__ nmoves) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= *nmoves) return;
  const int y = blockIdx.y;
  const int64_t h = hole_at[k], m = mover_at[k];
  switch (a.word[y]) {
    case 16: move_words<16>(a.base[y], a.stride[y], h, m); break;
    case 8: move_words<8>(a.base[y], a.stride[y], h, m); break;
    case 4: move_words<4>(a.base[y], a.stride[y], h, m); break;
    default: move_words<1>(a.base[y], a.stride[y], h, m); break;
  }
}

// Zero `bytes` bytes at p: single bytes up to the first 16-byte boundary,
// 16-byte stores for the aligned body, single bytes for the rest.
__global__ __launch_bounds__(256) void zero_kernel(char* __restrict__ p, int64_t head,
                                                   int64_t nbody, int64_t bytes) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < head) p[i] = 0;
  if (i < nbody) reinterpret_cast<uint4*>(p + head)[i] = make_uint4(0u, 0u, 0u, 0u);
  const int64_t tail0 = head + (nbody << 4);
  if (i < bytes - tail0) p[tail0 + i] = 0;
}

}  // namespace

int64_t container_tile_size() { return kTile; }

int64_t container_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

// 16-byte loads of the flags need a 16-byte aligned array.
static int flags_vec(const uint8_t* flags) { return (reinterpret_cast<uintptr_t>(flags) & 15u) == 0; }

hipError_t launch_count_flags(const uint8_t* flags, int64_t n, int32_t* counts, hipStream_t s) {
  const int64_t grid = container_tiles(n);
  if (grid > 0)
    hipLaunchKernelGGL(count_flags_kernel, dim3(grid), dim3(kBlock), 0, s, flags, n,
                       flags_vec(flags), counts);
  return hipGetLastError();
}

hipError_t launch_rank_flags(const uint8_t* flags, int64_t n, int64_t n_new,
                             const int64_t* holes_before, const int64_t* movers_after,
                             int64_t* hole_at, int64_t* mover_at, int64_t* nmoves, hipStream_t s) {
  const int64_t grid = container_tiles(n);
  if (grid > 0)
    hipLaunchKernelGGL(rank_kernel, dim3(grid), dim3(kBlock), 0, s, flags, n, flags_vec(flags),
                       n_new, holes_before, movers_after, hole_at, mover_at, nmoves);
  return hipGetLastError();
}

hipError_t launch_move_all(const MoveArgs& m, const int64_t* hole_at, const int64_t* mover_at,
                           const int64_t* nmoves, int64_t max_moves, hipStream_t s) {
  if (max_moves <= 0 || m.narrays <= 0) return hipSuccess;
  for (int y = 0; y < m.narrays; ++y) {
    const int w = m.word[y];
    if ((w != 1 && w != 4 && w != 8 && w != 16) || m.stride[y] % w) return hipErrorInvalidValue;
  }
  const int64_t grid = (max_moves + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(move_all_kernel, dim3(grid, m.narrays), dim3(kBlock), 0, s, m, hole_at,
                     mover_at, nmoves);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  const int64_t mis = static_cast<int64_t>(reinterpret_cast<uintptr_t>(p) & 15u);
  const int64_t head = std::min(bytes, (16 - mis) & 15);
  const int64_t nbody = (bytes - head) >> 4;
  const int64_t tail = bytes - head - (nbody << 4);  // < 16
  const int64_t threads = std::max(nbody, std::max(head, tail));
  const int64_t grid = (threads + 255) / 256;
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, s, static_cast<char*>(p), head, nbody,
                     bytes);
  return hipGetLastError();
}

}  // namespace soax
