// host_containers.cpp -- host side of the container calls: capacity,
// reserve, resize, push_back, rebind, element writes and removal by
// overwriting with the last particle.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host_internal.h"

using namespace soax;
using namespace soax::host;

// ----------------------------------------------------------- containers

namespace {

// Move an owned set into buffers for `cap` particles, keeping its n
// particles in both copies.  Synchronises `s` before freeing the old buffers.
soax_status grow(soax_set* set, int64_t cap, hipStream_t s) {
  void* nsoa_block = nullptr;
  void* naos = nullptr;
  std::vector<void*> nsoa;
  soax_status st = alloc_owned(set->L, cap, &nsoa_block, nsoa, &naos);
  if (st) return st;
  hipError_t e = hipSuccess;
  if (set->n > 0) {
    for (const Field& f : set->L.f)
      for (int c = 0; c < f.dim && e == hipSuccess; ++c) {
        const int a = f.first_array + c;
        e = launch_copy16(nsoa[a], set->soa[a], set->n * f.es, s);
      }
    if (e == hipSuccess) e = launch_copy16(naos, set->aos, set->n * set->L.stride, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(nsoa_block);
    (void)hipFree(naos);
    return hip_fail(e, "copy into the grown buffers");
  }
  (void)hipFree(set->owned_soa);
  (void)hipFree(set->owned_aos);
  set->owned_soa = nsoa_block;
  set->owned_aos = naos;
  set->soa = nsoa;
  set->aos = static_cast<char*>(naos);
  set->cap = cap;
  set->aosoa = nullptr;  // the AoSoA table names the old SoA arrays
  ++set->generation;
  return finish_set(set);  // the stream is idle: the new table can be uploaded
}

// Room for `need` particles: bound sets must already have it; owned sets
// grow to max(need, 2 * capacity), at most 2^31-1.
soax_status ensure_capacity(soax_set* set, int64_t need, hipStream_t s) {
  if (need <= set->cap) return SOAX_OK;
  if (!set->owns)
    return fail(SOAX_E_STATE, "a bound set holds at most %lld particles (asked for %lld)",
                static_cast<long long>(set->cap), static_cast<long long>(need));
  return grow(set, std::max(need, std::min(2 * set->cap, kMaxParticles)), s);
}

// New size (host state only: the kernels take n as an argument).
soax_status set_size(soax_set* set, int64_t n) {
  set->n = n;
  set->xpose_host.n = n;
  ++set->generation;
  return SOAX_OK;
}

// Pinned host scratch of at least `bytes`, once its last use has finished.
soax_status pinned_scratch(soax_set* set, size_t bytes, void** p) {
  if (set->pinned_pending) {
    HIP_TRY(hipEventSynchronize(set->pinned_done), "hipEventSynchronize");
    set->pinned_pending = false;
  }
  if (!set->pinned_done)
    HIP_TRY(hipEventCreateWithFlags(&set->pinned_done, hipEventDisableTiming), "hipEventCreate");
  if (set->pinned_bytes < bytes) {
    if (set->pinned) (void)hipHostFree(set->pinned);
    set->pinned = nullptr;
    set->pinned_bytes = 0;
    HIP_TRY(hipHostMalloc(&set->pinned, bytes, hipHostMallocDefault), "hipHostMalloc");
    set->pinned_bytes = bytes;
  }
  *p = set->pinned;
  return SOAX_OK;
}

// Width in bytes of the moves of one AoS record: the widest of 16, 8, 4
// that divides the stride and the buffer's alignment.
int record_word(const soax_set* set) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(set->aos);
  for (int w : {16, 8, 4})
    if (set->L.stride % w == 0 && a % w == 0) return w;
  return 1;
}

struct DevBuf {  // stream-ordered scratch, released on the same stream
  void* p = nullptr;
  hipStream_t s = nullptr;
  hipError_t alloc(size_t bytes, hipStream_t st) {
    s = st;
    return bytes ? hipMallocAsync(&p, bytes, st) : hipSuccess;
  }
  ~DevBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

}  // namespace

extern "C" {

soax_status soax_capacity(const soax_set* set, int64_t* n, int64_t* capacity) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (n) *n = set->n;
  if (capacity) *capacity = set->cap;
  return SOAX_OK;
}

soax_status soax_reserve(soax_set* set, int64_t capacity, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  soax_status st;
  if ((st = check_n(set->L, capacity))) return st;
  if (capacity <= set->cap) return SOAX_OK;
  const hipStream_t s = as_stream(stream);
  if (!set->owns)
    return fail(SOAX_E_STATE, "a bound set holds at most %lld particles",
                static_cast<long long>(set->cap));
  return grow(set, capacity, s);
}

soax_status soax_resize(soax_set* set, int64_t n, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  soax_status st;
  if ((st = check_n(set->L, n))) return st;
  const hipStream_t s = as_stream(stream);
  if ((st = ensure_capacity(set, n, s))) return st;
  if (n > set->n) {
    const int64_t add = n - set->n;
    if (has_soa(set))
      for (const Field& f : set->L.f)
        for (int c = 0; c < f.dim; ++c)
          HIP_TRY(launch_zero(static_cast<char*>(set->soa[f.first_array + c]) + set->n * f.es,
                              add * f.es, s),
                  "zero fill launch");
    if (set->aos)
      HIP_TRY(launch_zero(set->aos + set->n * set->L.stride, add * set->L.stride, s),
              "zero fill launch");
  }
  return set_size(set, n);
}

soax_status soax_push_back(soax_set* set, const void* host_records, int64_t count, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (count < 0) return fail(SOAX_E_ARG, "count is negative");
  if (count > 0 && !host_records) return fail(SOAX_E_ARG, "host_records is NULL");
  soax_status st;
  if ((st = check_n(set->L, set->n + count))) return st;
  if (has_soa(set) && !set->owns && !set->soa_vec_ok)
    return fail(SOAX_E_LAYOUT, "push_back needs 16-byte aligned SoA arrays");
  const hipStream_t s = as_stream(stream);
  if ((st = ensure_capacity(set, set->n + count, s))) return st;
  if (count == 0) return SOAX_OK;
  const Layout& L = set->L;
  const int64_t n0 = set->n;
  const int64_t bytes = count * L.stride;
  {
    DevBuf stage, table;
    HIP_TRY(stage.alloc(bytes, s), "hipMallocAsync(staging)");
    HIP_TRY(hipMemcpyAsync(stage.p, host_records, bytes, hipMemcpyHostToDevice, s),
            "hipMemcpyAsync(records)");
    XposeArgs t = set->xpose_host;  // same fields; the appended range only
    if (has_soa(set)) {
      t.aos = static_cast<char*>(stage.p);
      t.n = count;
      t.stride = static_cast<int32_t>(L.stride);
      t.narrays = L.narrays;
      t.aligned = 1;
      for (const Field& f : L.f) {
        if (f.off % f.es || L.stride % f.es) t.aligned = 0;
        for (int c = 0; c < f.dim; ++c) {
          const int a = f.first_array + c;
          t.soa[a] = static_cast<char*>(set->soa[a]) + n0 * f.es;
          t.off[a] = static_cast<int32_t>(f.off + c * f.es);
          t.es[a] = f.es;
        }
      }
      group_by_size(t);
      HIP_TRY(table.alloc(sizeof(XposeArgs), s), "hipMallocAsync(table)");
      HIP_TRY(hipMemcpyAsync(table.p, &t, sizeof(XposeArgs), hipMemcpyHostToDevice, s),
              "hipMemcpyAsync(table)");
      HIP_TRY(launch_xpose(true, t, static_cast<const XposeArgs*>(table.p), s), "transpose launch");
    }
    if (set->aos)
      HIP_TRY(hipMemcpyAsync(set->aos + n0 * L.stride, stage.p, bytes, hipMemcpyDeviceToDevice, s),
              "hipMemcpyAsync(records)");
    // the host records and the host table must outlive the copies
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  return set_size(set, n0 + count);
}

soax_status soax_rebind(soax_set* set, int64_t capacity, void* const* soa_ptrs, void* aos_ptr,
                        void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (set->owns) return fail(SOAX_E_STATE, "the set owns its buffers (use soax_reserve)");
  soax_status st;
  if ((st = check_n(set->L, capacity))) return st;
  if (capacity < set->n)
    return fail(SOAX_E_ARG, "capacity %lld is below n = %lld", static_cast<long long>(capacity),
                static_cast<long long>(set->n));
  if (has_soa(set) != (soa_ptrs != nullptr) || has_aos(set) != (aos_ptr != nullptr))
    return fail(SOAX_E_LAYOUT, "the new buffers must give the same copies as the old ones");
  if (capacity > 0 && soa_ptrs)
    for (int a = 0; a < set->L.narrays; ++a)
      if (!soa_ptrs[a]) return fail(SOAX_E_ARG, "soa_ptrs[%d] is NULL", a);
  const hipStream_t s = as_stream(stream);
  auto move = [&](void* dst, const void* src, int64_t bytes) {
    if (bytes == 0) return hipSuccess;
    if (aligned16(dst) && aligned16(src)) return launch_copy16(dst, src, bytes, s);
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
  };
  if (set->n > 0) {
    if (soa_ptrs)
      for (const Field& f : set->L.f)
        for (int c = 0; c < f.dim; ++c) {
          const int a = f.first_array + c;
          HIP_TRY(move(soa_ptrs[a], set->soa[a], set->n * f.es), "copy into the new buffers");
        }
    if (aos_ptr)
      HIP_TRY(move(aos_ptr, set->aos, set->n * set->L.stride), "copy into the new buffers");
  }
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");  // copies done, old table unused
  if (soa_ptrs) set->soa.assign(soa_ptrs, soa_ptrs + set->L.narrays);
  set->aos = static_cast<char*>(aos_ptr);
  set->cap = capacity;
  set->aosoa = nullptr;  // the AoSoA table names the old SoA arrays
  ++set->generation;
  return finish_set(set);
}

soax_status soax_set_record(soax_set* set, int64_t i, const void* host_record) {
  if (!set || !host_record) return fail(SOAX_E_ARG, "set or host_record is NULL");
  if (i < 0 || i >= set->n) return fail(SOAX_E_ARG, "record %lld out of range", static_cast<long long>(i));
  const Layout& L = set->L;
  const char* in = static_cast<const char*>(host_record);
  if (set->aos)
    HIP_TRY(hipMemcpy(set->aos + i * L.stride, in, L.stride, hipMemcpyHostToDevice), "hipMemcpy");
  if (has_soa(set))
    for (const Field& f : L.f)
      for (int c = 0; c < f.dim; ++c)
        HIP_TRY(hipMemcpy(static_cast<char*>(set->soa[f.first_array + c]) + i * f.es,
                          in + f.off + c * f.es, f.es, hipMemcpyHostToDevice),
                "hipMemcpy");
  return SOAX_OK;
}

soax_status soax_remove_flagged(soax_set* set, const uint8_t* flags, int64_t* new_n, void* stream) {
  if (!set || !new_n) return fail(SOAX_E_ARG, "set or new_n is NULL");
  const int64_t n = set->n;
  if (n > 0 && !flags) return fail(SOAX_E_ARG, "flags is NULL");
  *new_n = n;
  if (n == 0) return SOAX_OK;
  const hipStream_t s = as_stream(stream);
  const int64_t tiles = container_tiles(n);
  // pinned staging: tile counts (int32), then the two offset tables (int64)
  const size_t counts_bytes = (tiles * sizeof(int32_t) + 15) & ~size_t(15);
  void* host = nullptr;
  soax_status st;
  if ((st = pinned_scratch(set, counts_bytes + 2 * tiles * sizeof(int64_t), &host))) return st;
  int32_t* counts = static_cast<int32_t*>(host);
  int64_t* tab = reinterpret_cast<int64_t*>(static_cast<char*>(host) + counts_bytes);
  DevBuf dcounts;
  HIP_TRY(dcounts.alloc(tiles * sizeof(int32_t), s), "hipMallocAsync(counts)");
  int32_t* dc = static_cast<int32_t*>(dcounts.p);
  HIP_TRY(launch_count_flags(flags, n, dc, s), "flag count launch");
  HIP_TRY(hipMemcpyAsync(counts, dc, tiles * sizeof(int32_t), hipMemcpyDeviceToHost, s),
          "hipMemcpyAsync(counts)");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");  // the one wait: n' is returned
  int64_t m = 0;
  for (int64_t b = 0; b < tiles; ++b) m += counts[b];
  const int64_t n_new = n - m;
  const int64_t moves_max = std::min(m, n_new);
  if (moves_max > 0) {
    // tab[b]: flagged in tiles < b; tab[tiles + b]: unflagged in tiles > b
    const int64_t T = container_tile_size();
    int64_t acc = 0;
    for (int64_t b = 0; b < tiles; ++b) {
      tab[b] = acc;
      acc += counts[b];
    }
    acc = 0;
    for (int64_t b = tiles - 1; b >= 0; --b) {
      tab[tiles + b] = acc;
      acc += std::min(T, n - b * T) - counts[b];
    }
    MoveArgs mv{};
    if (has_soa(set))
      for (const Field& f : set->L.f)
        for (int c = 0; c < f.dim; ++c) {
          mv.base[mv.narrays] = static_cast<char*>(set->soa[f.first_array + c]);
          mv.stride[mv.narrays] = f.es;
          mv.word[mv.narrays] = f.es;
          ++mv.narrays;
        }
    if (set->aos) {
      mv.base[mv.narrays] = set->aos;
      mv.stride[mv.narrays] = static_cast<int32_t>(set->L.stride);
      mv.word[mv.narrays] = record_word(set);
      ++mv.narrays;
    }
    DevBuf dtab, dlists;
    HIP_TRY(dtab.alloc(2 * tiles * sizeof(int64_t), s), "hipMallocAsync(offsets)");
    HIP_TRY(dlists.alloc((2 * moves_max + 1) * sizeof(int64_t), s), "hipMallocAsync(lists)");
    int64_t* dt = static_cast<int64_t*>(dtab.p);
    int64_t* hole_at = static_cast<int64_t*>(dlists.p);
    int64_t* mover_at = hole_at + moves_max;
    int64_t* nmoves = mover_at + moves_max;
    HIP_TRY(hipMemcpyAsync(dt, tab, 2 * tiles * sizeof(int64_t), hipMemcpyHostToDevice, s),
            "hipMemcpyAsync(offsets)");
    HIP_TRY(hipEventRecord(set->pinned_done, s), "hipEventRecord");
    set->pinned_pending = true;
    HIP_TRY(launch_rank_flags(flags, n, n_new, dt, dt + tiles, hole_at, mover_at, nmoves, s),
            "rank launch");
    HIP_TRY(launch_move_all(mv, hole_at, mover_at, nmoves, moves_max, s), "move launch");
  }
  *new_n = n_new;
  return set_size(set, n_new);
}

}  // extern "C"
