// host_internal.h -- what the host-side translation units of the C ABI
// share: error reporting, the parsed schema and record layout, the particle
// set handle and its buffer helpers.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "launch.h"
#include "soax.h"

namespace soax {
namespace host {

// Record a thread-local message for soax_last_error and return st.
soax_status fail(soax_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
soax_status hip_fail(hipError_t e, const char* what);
const char* last_error();

inline bool is_finite(double x) { return isfinite(x) != 0; }
inline bool is_real(int32_t t) { return t == kF32 || t == kF64; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

constexpr int64_t kMaxParticles = INT32_MAX;

struct Field {
  std::string name;
  int32_t dtype;
  int32_t dim;
  char tag;
  int64_t off;       // AoS byte offset
  int es;            // element size
  int first_array;   // index of component 0 in the SoA array list
};

struct Layout {
  std::vector<Field> f;
  int32_t packed = 0;
  int64_t stride = 0;
  int64_t soa_bytes = 0;
  int narrays = 0;

  int find(const char* name) const {
    for (size_t i = 0; i < f.size(); ++i)
      if (f[i].name == name) return static_cast<int>(i);
    return -1;
  }
};

// C struct rule: each member at the next multiple of its alignment (for
// these scalar types, its size), the record padded to a multiple of the
// largest member alignment.  Packed: members back to back.
soax_status parse_schema(const soax_schema* s, Layout& L);
// A 3-vector float property, or an error recorded.
soax_status vec_field(const Layout& L, const char* name, int* idx);

}  // namespace host
}  // namespace soax

#define HIP_TRY(call, what)                                         \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return soax::host::hip_fail(e_, what);    \
  } while (0)

struct soax_set {
  soax::host::Layout L;
  int64_t n = 0;
  int64_t cap = 0;         // particles every buffer can hold
  uint64_t generation = 0; // bumped whenever n or a buffer address changes
  std::vector<void*> soa;  // one per array; empty if there is no SoA copy
  char* aos = nullptr;
  bool owns = false;       // buffers allocated (and grown) by the library
  void* owned_soa = nullptr;
  void* owned_aos = nullptr;
  bool soa_vec_ok = false;    // every SoA array 16-byte aligned
  bool aos_base_ok = false;   // AoS buffer 16-byte aligned
  soax::XposeArgs* xpose_dev = nullptr;
  soax::XposeArgs xpose_host{};
  int block[4] = {0, 0, 0, 0};
  int vec = 0;
  // optional AoSoA copy (caller-owned buffer) and its conversion table
  char* aosoa = nullptr;
  int64_t aosoa_bytes = 0;
  soax::XposeArgs* aosoa_dev = nullptr;
  soax::XposeArgs aosoa_host{};
  // pinned host staging of the removal's tile counts and offsets, reused
  // once the event says the last copy out of it has finished
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_done = nullptr;
  bool pinned_pending = false;
};

namespace soax {
namespace host {

soax_status check_n(const Layout& L, int64_t n);
// An owned set always has both copies (its buffers are null while it holds
// room for no particle); a bound set has the copies it was given.
inline bool has_soa(const soax_set* s) { return !s->soa.empty(); }
inline bool has_aos(const soax_set* s) { return s->owns || s->aos != nullptr; }
// AoSoA: byte offset of every SoA array inside a tile, and bytes per tile.
int64_t aosoa_tile(const Layout& L, std::vector<int32_t>* off);
int64_t aosoa_need(const Layout& L, int64_t cap);
// Fill the transpose table from the set's buffers and size, and upload it
// (synchronous copy; callers order it after earlier work that reads it).
soax_status finish_set(soax_set* s);
// Library-owned buffers for `cap` particles: one allocation holding every
// SoA array on its own 256-byte boundary, and the AoS records.
soax_status alloc_owned(const Layout& L, int64_t cap, void** soa_block, std::vector<void*>& soa,
                        void** aos);
void free_set(soax_set* s);

}  // namespace host
}  // namespace soax
