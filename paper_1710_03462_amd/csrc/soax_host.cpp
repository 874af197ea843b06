// soax_host.cpp -- host side of the C ABI declared in include/soax.h:
// schema validation and record layout, particle-set handles, argument
// checks (all done before any device call), kernel dispatch, the batched
// stepping with its hipGraph cache, and the autotuner.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "launch.h"
#include "soax.h"

using namespace soax;

namespace {

thread_local std::string g_last_error;

soax_status fail(soax_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

soax_status hip_fail(hipError_t e, const char* what) {
  return fail(SOAX_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_finite(double x) { return isfinite(x) != 0; }

constexpr int64_t kMaxParticles = INT32_MAX;

// ------------------------------------------------------------------ schema

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
soax_status parse_schema(const soax_schema* s, Layout& L) {
  if (!s) return fail(SOAX_E_ARG, "schema is NULL");
  if (!s->fields) return fail(SOAX_E_ARG, "schema.fields is NULL");
  if (s->nfields < 1 || s->nfields > kMaxFields)
    return fail(SOAX_E_SCHEMA, "nfields %d outside 1..%d", s->nfields, kMaxFields);
  if (s->packed != 0 && s->packed != 1) return fail(SOAX_E_ARG, "packed must be 0 or 1");
  L = Layout();
  L.packed = s->packed;
  int64_t end = 0, maxal = 1;
  int arrays = 0;
  for (int i = 0; i < s->nfields; ++i) {
    const soax_field& fd = s->fields[i];
    if (!fd.name) return fail(SOAX_E_SCHEMA, "field %d has no name", i);
    const size_t len = strnlen(fd.name, 64);
    if (len == 0 || len > 31) return fail(SOAX_E_SCHEMA, "field %d name length must be 1..31", i);
    const int es = dtype_size(fd.dtype);
    if (es == 0) return fail(SOAX_E_SCHEMA, "field '%s' has unknown dtype %d", fd.name, fd.dtype);
    if (fd.dim < 1 || fd.dim > 3) return fail(SOAX_E_SCHEMA, "field '%s' dim %d outside 1..3", fd.name, fd.dim);
    for (const Field& g : L.f)
      if (g.name == fd.name) return fail(SOAX_E_SCHEMA, "duplicate field name '%s'", fd.name);
    if (!L.packed && end % es) end += es - end % es;
    Field f{fd.name, fd.dtype, fd.dim, fd.tag, end, es, arrays};
    L.f.push_back(f);
    end += static_cast<int64_t>(es) * fd.dim;
    L.soa_bytes += static_cast<int64_t>(es) * fd.dim;
    arrays += fd.dim;
    if (es > maxal) maxal = es;
  }
  if (!L.packed && end % maxal) end += maxal - end % maxal;
  L.stride = end;
  L.narrays = arrays;
  return SOAX_OK;
}

bool is_real(int32_t t) { return t == kF32 || t == kF64; }

// A 3-vector float property, or -1 with an error recorded.
soax_status vec_field(const Layout& L, const char* name, int* idx) {
  const int f = L.find(name);
  if (f < 0) return fail(SOAX_E_SCHEMA, "schema has no '%s' property", name);
  if (L.f[f].dim != 3 || !is_real(L.f[f].dtype))
    return fail(SOAX_E_SCHEMA, "'%s' must be a 3-component f32/f64 property", name);
  *idx = f;
  return SOAX_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

// ----------------------------------------------------------------- the set

struct soax_set {
  Layout L;
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
  XposeArgs* xpose_dev = nullptr;
  XposeArgs xpose_host{};
  int block[4] = {0, 0, 0, 0};
  int vec = 0;
  // optional AoSoA copy (caller-owned buffer) and its conversion table
  char* aosoa = nullptr;
  int64_t aosoa_bytes = 0;
  XposeArgs* aosoa_dev = nullptr;
  XposeArgs aosoa_host{};
  // pinned host staging of the removal's tile counts and offsets, reused
  // once the event says the last copy out of it has finished
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_done = nullptr;
  bool pinned_pending = false;
};

struct soax_batch {
  std::vector<soax_set*> sets;
  std::vector<uint64_t> generations;  // of each set when the batch was made
  int vel_t = kF32;
  int64_t total = 0;
  int block = 256, per_thread = 2, blocks_per_cu = 8;
  int cus = 256;
  std::string arch;
  // device tables
  BatchSet* dev_sets = nullptr;
  int32_t* dev_tile_set = nullptr;
  int64_t ntiles = 0;
  int tile_for = 0;  // tile size the tile list was built for
  // host staging of the set table (pinned) and the event guarding its reuse
  BatchSet* stage = nullptr;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
  hipStream_t capture_stream = nullptr;
  std::map<std::tuple<int64_t, int, int, int>, hipGraphExec_t> graphs;
};

struct soax_step_graph {
  soax_set* set = nullptr;
  uint64_t generation = 0;  // of the set when captured
  hipGraphExec_t exec = nullptr;
};

namespace {

soax_status check_n(const Layout& L, int64_t n) {
  if (n < 0) return fail(SOAX_E_ARG, "n = %lld is negative", static_cast<long long>(n));
  if (n > kMaxParticles)
    return fail(SOAX_E_RANGE, "n = %lld exceeds 2^31-1 records", static_cast<long long>(n));
  const int fid = L.find("id");
  if (fid >= 0 && ((L.f[fid].dtype == kI8 && n > 128) || (L.f[fid].dtype == kU8 && n > 256) ||
                   (L.f[fid].dtype == kI32 && n > INT32_MAX)))
    return fail(SOAX_E_RANGE, "the 'id' type cannot number %lld particles", static_cast<long long>(n));
  return SOAX_OK;
}

// An owned set always has both copies (its buffers are null while it holds
// room for no particle); a bound set has the copies it was given.
bool has_soa(const soax_set* s) { return !s->soa.empty(); }
bool has_aos(const soax_set* s) { return s->owns || s->aos != nullptr; }

// AoSoA: byte offset of every SoA array inside a tile, and bytes per tile.
int64_t aosoa_tile(const Layout& L, std::vector<int32_t>* off) {
  int64_t acc = 0;
  if (off) off->assign(L.narrays, 0);
  for (const Field& f : L.f)
    for (int c = 0; c < f.dim; ++c) {
      if (off) (*off)[f.first_array + c] = static_cast<int32_t>(kAosoaW * acc);
      acc += f.es;
    }
  return kAosoaW * acc;
}

int64_t aosoa_need(const Layout& L, int64_t cap) {
  return (cap + kAosoaW - 1) / kAosoaW * aosoa_tile(L, nullptr);
}

// Fill the transpose table from the set's buffers and size, and upload it
// (synchronous copy; callers order it after earlier work that reads it).
soax_status finish_set(soax_set* s) {
  s->soa_vec_ok = !s->soa.empty();
  for (void* p : s->soa)
    if (!aligned16(p)) s->soa_vec_ok = false;
  s->aos_base_ok = s->aos ? aligned16(s->aos) : s->owns;
  XposeArgs& t = s->xpose_host;
  t.aos = s->aos;
  t.n = s->n;
  t.stride = static_cast<int32_t>(s->L.stride);
  t.narrays = s->L.narrays;
  t.aligned = 1;
  for (const Field& f : s->L.f) {
    if (f.off % f.es || s->L.stride % f.es) t.aligned = 0;
    for (int c = 0; c < f.dim; ++c) {
      const int a = f.first_array + c;
      t.soa[a] = s->soa.empty() ? nullptr : static_cast<char*>(s->soa[a]);
      t.off[a] = static_cast<int32_t>(f.off + c * f.es);
      t.es[a] = f.es;
    }
  }
  if (s->cap > 0 && has_soa(s) && has_aos(s)) {
    if (!s->xpose_dev) {
      void* d = nullptr;
      hipError_t e = hipMalloc(&d, sizeof(XposeArgs));
      if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(transpose table): %s", hipGetErrorString(e));
      s->xpose_dev = static_cast<XposeArgs*>(d);
    }
    HIP_TRY(hipMemcpy(s->xpose_dev, &t, sizeof(XposeArgs), hipMemcpyHostToDevice),
            "hipMemcpy(transpose table)");
  }
  return SOAX_OK;
}

// Library-owned buffers for `cap` particles: one allocation holding every
// SoA array on its own 256-byte boundary, and the AoS records.
soax_status alloc_owned(const Layout& L, int64_t cap, void** soa_block, std::vector<void*>& soa,
                        void** aos) {
  *soa_block = nullptr;
  *aos = nullptr;
  soa.assign(L.narrays, nullptr);
  if (cap == 0) return SOAX_OK;
  std::vector<int64_t> off(L.narrays);
  int64_t total = 0;
  for (const Field& f : L.f)
    for (int c = 0; c < f.dim; ++c) {
      off[f.first_array + c] = total;
      total += (cap * f.es + 255) & ~int64_t(255);
    }
  hipError_t e = hipMalloc(soa_block, total);
  if (e != hipSuccess) {
    *soa_block = nullptr;
    return fail(SOAX_E_OOM, "hipMalloc(%lld bytes for SoA): %s", static_cast<long long>(total),
                hipGetErrorString(e));
  }
  for (int a = 0; a < L.narrays; ++a) soa[a] = static_cast<char*>(*soa_block) + off[a];
  e = hipMalloc(aos, cap * L.stride);
  if (e != hipSuccess) {
    (void)hipFree(*soa_block);
    *soa_block = nullptr;
    *aos = nullptr;
    return fail(SOAX_E_OOM, "hipMalloc(%lld bytes for AoS): %s",
                static_cast<long long>(cap * L.stride), hipGetErrorString(e));
  }
  return SOAX_OK;
}

void free_set(soax_set* s) {
  if (!s) return;
  if (s->aosoa_dev) (void)hipFree(s->aosoa_dev);
  if (s->pinned_pending) (void)hipEventSynchronize(s->pinned_done);
  if (s->pinned_done) (void)hipEventDestroy(s->pinned_done);
  if (s->pinned) (void)hipHostFree(s->pinned);
  if (s->xpose_dev) (void)hipFree(s->xpose_dev);
  if (s->owned_soa) (void)hipFree(s->owned_soa);
  if (s->owned_aos) (void)hipFree(s->owned_aos);
  delete s;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

soax_status soax_schema_layout(const soax_schema* schema, int64_t* offsets, int64_t* stride,
                               int64_t* soa_bytes) {
  Layout L;
  soax_status st = parse_schema(schema, L);
  if (st) return st;
  if (offsets)
    for (size_t i = 0; i < L.f.size(); ++i) offsets[i] = L.f[i].off;
  if (stride) *stride = L.stride;
  if (soa_bytes) *soa_bytes = L.soa_bytes;
  return SOAX_OK;
}

soax_status soax_create(const soax_schema* schema, int64_t n, soax_set** out) {
  if (!out) return fail(SOAX_E_ARG, "out is NULL");
  *out = nullptr;
  Layout L;
  soax_status st = parse_schema(schema, L);
  if (st) return st;
  if ((st = check_n(L, n))) return st;
  soax_set* s = new soax_set();
  s->L = L;
  s->n = n;
  s->cap = n;
  s->owns = true;
  if ((st = alloc_owned(L, n, &s->owned_soa, s->soa, &s->owned_aos))) {
    free_set(s);
    return st;
  }
  s->aos = static_cast<char*>(s->owned_aos);
  if ((st = finish_set(s))) {
    free_set(s);
    return st;
  }
  *out = s;
  return SOAX_OK;
}

soax_status soax_bind_capacity(const soax_schema* schema, int64_t n, int64_t capacity,
                               void* const* soa_ptrs, void* aos_ptr, soax_set** out) {
  if (!out) return fail(SOAX_E_ARG, "out is NULL");
  *out = nullptr;
  Layout L;
  soax_status st = parse_schema(schema, L);
  if (st) return st;
  if ((st = check_n(L, n)) || (st = check_n(L, capacity))) return st;
  if (capacity < n) return fail(SOAX_E_ARG, "capacity %lld is below n = %lld",
                                static_cast<long long>(capacity), static_cast<long long>(n));
  if (!soa_ptrs && !aos_ptr) return fail(SOAX_E_ARG, "neither a SoA nor an AoS buffer was given");
  if (capacity > 0 && soa_ptrs)
    for (int a = 0; a < L.narrays; ++a)
      if (!soa_ptrs[a]) return fail(SOAX_E_ARG, "soa_ptrs[%d] is NULL", a);
  soax_set* s = new soax_set();
  s->L = L;
  s->n = n;
  s->cap = capacity;
  if (soa_ptrs) s->soa.assign(soa_ptrs, soa_ptrs + L.narrays);
  s->aos = static_cast<char*>(aos_ptr);
  if ((st = finish_set(s))) {
    free_set(s);
    return st;
  }
  *out = s;
  return SOAX_OK;
}

soax_status soax_bind(const soax_schema* schema, int64_t n, void* const* soa_ptrs, void* aos_ptr,
                      soax_set** out) {
  return soax_bind_capacity(schema, n, n, soa_ptrs, aos_ptr, out);
}

void soax_destroy(soax_set* set) { free_set(set); }

soax_status soax_layout_info(const soax_set* set, int64_t* offsets, int64_t* stride,
                             int64_t* soa_bytes) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (offsets)
    for (size_t i = 0; i < set->L.f.size(); ++i) offsets[i] = set->L.f[i].off;
  if (stride) *stride = set->L.stride;
  if (soa_bytes) *soa_bytes = set->L.soa_bytes;
  return SOAX_OK;
}

soax_status soax_buffer(const soax_set* set, int32_t index, void** ptr) {
  if (!set || !ptr) return fail(SOAX_E_ARG, "set or ptr is NULL");
  if (index == -1) {
    *ptr = set->aos;
    return SOAX_OK;
  }
  if (index == -2) {
    *ptr = set->aosoa;
    return SOAX_OK;
  }
  if (index < 0 || index >= set->L.narrays) return fail(SOAX_E_ARG, "array index %d out of range", index);
  *ptr = set->soa.empty() ? nullptr : set->soa[index];
  return SOAX_OK;
}

soax_status soax_fill(soax_set* set, uint64_t seed, int32_t vel_mode, const soax_params* params,
                      void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (vel_mode != 0 && vel_mode != 1) return fail(SOAX_E_ARG, "vel_mode must be 0 or 1");
  if (set->soa.empty()) return fail(SOAX_E_LAYOUT, "the set has no SoA copy to fill");
  const Layout& L = set->L;
  int fpos = -1, fvel = -1;
  if (vel_mode == 1) {
    soax_status st;
    if ((st = vec_field(L, "pos", &fpos)) || (st = vec_field(L, "vel", &fvel))) return st;
    if (!params || !is_finite(params->A) || !is_finite(params->B) || !is_finite(params->C))
      return fail(SOAX_E_ARG, "vel_mode 1 needs finite field amplitudes");
  }
  hipStream_t s = as_stream(stream);
  for (size_t fi = 0; fi < L.f.size(); ++fi) {
    const Field& f = L.f[fi];
    if (static_cast<int>(fi) == fvel) continue;
    const bool real = is_real(f.dtype);
    int rule;
    if (f.name == "id") rule = kFillIndex;
    else if (f.name == "pos" && real) rule = kFillBox;
    else if ((f.name == "vel" || f.name == "acc") && real) rule = kFillNormal;
    else if (f.name == "mass" && real) rule = kFillMass;
    else if (f.name == "flags" && !real) rule = kFillTop8;
    else rule = real ? kFillUnit : kFillRaw;
    for (int c = 0; c < f.dim; ++c) {
      FillArgs a{set->soa[f.first_array + c], set->n, seed,
                 8 * static_cast<uint64_t>(fi) + 2 * static_cast<uint64_t>(c), f.dtype, rule};
      HIP_TRY(launch_fill(a, s), "fill kernel launch");
    }
  }
  if (vel_mode == 1) {
    SoaStepArgs a{};
    for (int d = 0; d < 3; ++d) {
      a.pos[d] = set->soa[L.f[fpos].first_array + d];
      a.vel[d] = set->soa[L.f[fvel].first_array + d];
    }
    a.n = set->n;
    a.abc = AbcParams{params->A, params->B, params->C};
    HIP_TRY(launch_vel_from_field(L.f[fpos].dtype, L.f[fvel].dtype, a, s), "field fill launch");
  }
  return SOAX_OK;
}

soax_status soax_step_config(soax_set* set, int32_t layout, int32_t block, int32_t per_thread) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (layout < SOAX_SOA || layout > SOAX_AOSOA) return fail(SOAX_E_ARG, "unknown layout %d", layout);
  if (block != 0 && (block < 64 || block > 1024 || block % 64))
    return fail(SOAX_E_ARG, "block %d must be 0 or a multiple of 64 in 64..1024", block);
  if (per_thread != 0 && per_thread != 1 && per_thread != 2 && per_thread != 4)
    return fail(SOAX_E_ARG, "per_thread %d must be 0, 1, 2 or 4", per_thread);
  if (per_thread != 0 && layout != SOAX_SOA)
    return fail(SOAX_E_ARG, "per_thread applies to the SoA layout only");
  set->block[layout] = block;
  if (layout == SOAX_SOA) set->vec = per_thread;
  return SOAX_OK;
}

soax_status soax_step(soax_set* set, int32_t layout, int32_t integrator, double dt, int64_t nsteps,
                      const soax_params* params, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (layout < SOAX_SOA || layout > SOAX_AOSOA) return fail(SOAX_E_ARG, "unknown layout %d", layout);
  if (integrator < SOAX_EULER || integrator > SOAX_SYMPLECTIC_EULER)
    return fail(SOAX_E_ARG, "unknown integrator %d", integrator);
  if (!is_finite(dt)) return fail(SOAX_E_ARG, "dt is not finite");
  if (nsteps < 0) return fail(SOAX_E_ARG, "nsteps is negative");
  const Layout& L = set->L;
  int fp, fv, fa = -1;
  soax_status st;
  if ((st = vec_field(L, "pos", &fp)) || (st = vec_field(L, "vel", &fv))) return st;
  if (uses_acc(integrator)) {
    if ((st = vec_field(L, "acc", &fa))) return st;
    if (L.f[fa].dtype != L.f[fv].dtype)
      return fail(SOAX_E_SCHEMA, "'acc' must have the same type as 'vel'");
  }
  const int wrap = params ? params->wrap : 0;
  if (wrap != 0 && wrap != 1) return fail(SOAX_E_ARG, "params.wrap must be 0 or 1");
  AbcParams abc{0.0, 0.0, 0.0};
  if (field_integrator(integrator)) {
    if (!params) return fail(SOAX_E_ARG, "integrating in the ABC field needs params");
    if (L.f[fp].dtype != kF64) return fail(SOAX_E_SCHEMA, "integrating in the ABC field needs f64 'pos'");
  }
  if (params) {
    if (!is_finite(params->A) || !is_finite(params->B) || !is_finite(params->C))
      return fail(SOAX_E_ARG, "field amplitudes must be finite");
    abc = AbcParams{params->A, params->B, params->C};
  }
  if (wrap && L.f[fp].dtype != kF64) return fail(SOAX_E_SCHEMA, "the periodic wrap needs f64 'pos'");
  hipStream_t s = as_stream(stream);
  if (layout == SOAX_SOA) {
    if (set->soa.empty()) return fail(SOAX_E_LAYOUT, "the set has no SoA copy");
    SoaStepArgs a{};
    for (int d = 0; d < 3; ++d) {
      a.pos[d] = set->soa[L.f[fp].first_array + d];
      a.vel[d] = set->soa[L.f[fv].first_array + d];
      a.acc[d] = fa >= 0 ? set->soa[L.f[fa].first_array + d] : nullptr;
    }
    a.n = set->n;
    a.dt = dt;
    a.abc = abc;
    a.wrap = wrap;
    // one particle per thread in workgroups of 128: the fastest shape measured
    // on the MI355X for both the streaming Euler and the VALU-heavy RK2 step
    int vec = set->vec ? set->vec : 1;
    if (!set->soa_vec_ok) vec = 1;
    const int block = set->block[SOAX_SOA] ? set->block[SOAX_SOA] : 128;
    for (int64_t k = 0; k < nsteps; ++k)
      HIP_TRY(launch_soa_step(integrator, L.f[fp].dtype, L.f[fv].dtype, vec, block, a, s),
              "SoA step launch");
    return SOAX_OK;
  }
  if (layout == SOAX_AOSOA) {
    if (!set->aosoa) return fail(SOAX_E_LAYOUT, "the set has no AoSoA copy");
    std::vector<int32_t> off;
    AosoaStepArgs a{};
    a.base = set->aosoa;
    a.tile_bytes = aosoa_tile(L, &off);
    for (int d = 0; d < 3; ++d) {
      a.off_pos[d] = off[L.f[fp].first_array + d];
      a.off_vel[d] = off[L.f[fv].first_array + d];
      a.off_acc[d] = fa >= 0 ? off[L.f[fa].first_array + d] : 0;
    }
    a.n = set->n;
    a.dt = dt;
    a.abc = abc;
    a.wrap = wrap;
    const int block = set->block[SOAX_AOSOA] ? set->block[SOAX_AOSOA] : 128;
    for (int64_t k = 0; k < nsteps; ++k)
      HIP_TRY(launch_aosoa_step(integrator, L.f[fp].dtype, L.f[fv].dtype, block, a, s),
              "AoSoA step launch");
    return SOAX_OK;
  }
  if (!has_aos(set)) return fail(SOAX_E_LAYOUT, "the set has no AoS copy");
  AosStepArgs a{};
  a.aos = set->aos;
  a.n = set->n;
  a.stride = static_cast<int32_t>(L.stride);
  a.off_pos = static_cast<int32_t>(L.f[fp].off);
  a.off_vel = static_cast<int32_t>(L.f[fv].off);
  a.off_acc = fa >= 0 ? static_cast<int32_t>(L.f[fa].off) : 0;
  a.dt = dt;
  a.abc = abc;
  a.wrap = wrap;
  bool aligned = L.f[fp].off % L.f[fp].es == 0 && L.f[fv].off % L.f[fv].es == 0 &&
                 L.stride % L.f[fp].es == 0 && L.stride % L.f[fv].es == 0 &&
                 (fa < 0 || L.f[fa].off % L.f[fa].es == 0);
  if (reinterpret_cast<uintptr_t>(set->aos) % 8) aligned = false;
  if (layout == SOAX_AOS) {
    if (!set->aos_base_ok) return fail(SOAX_E_LAYOUT, "the AoS buffer is not 16-byte aligned");
    const int block = set->block[SOAX_AOS] ? set->block[SOAX_AOS] : 256;
    for (int64_t k = 0; k < nsteps; ++k)
      HIP_TRY(launch_aos_step(integrator, L.f[fp].dtype, L.f[fv].dtype, aligned, block, a, s),
              "AoS step launch");
  } else {
    const int block = set->block[SOAX_AOS_NAIVE] ? set->block[SOAX_AOS_NAIVE] : 256;
    for (int64_t k = 0; k < nsteps; ++k)
      HIP_TRY(launch_aos_naive(integrator, L.f[fp].dtype, L.f[fv].dtype, aligned, block, a, s),
              "naive AoS step launch");
  }
  return SOAX_OK;
}

static soax_status xpose(soax_set* set, bool to_soa, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (!has_soa(set) || !has_aos(set)) return fail(SOAX_E_LAYOUT, "the transpose needs both copies");
  if (!set->soa_vec_ok || !set->aos_base_ok)
    return fail(SOAX_E_LAYOUT, "the transpose needs 16-byte aligned buffers");
  if (set->n == 0) return SOAX_OK;
  HIP_TRY(launch_xpose(to_soa, set->xpose_host, set->xpose_dev, as_stream(stream)),
          "transpose launch");
  return SOAX_OK;
}

soax_status soax_aos_to_soa(soax_set* set, void* stream) { return xpose(set, true, stream); }
soax_status soax_soa_to_aos(soax_set* set, void* stream) { return xpose(set, false, stream); }

soax_status soax_step_graph_create(soax_set* set, int32_t layout, int32_t integrator, double dt,
                                   int64_t nsteps, const soax_params* params,
                                   soax_step_graph** out) {
  if (!out) return fail(SOAX_E_ARG, "out is NULL");
  *out = nullptr;
  // every argument check of soax_step, with nothing launched
  soax_status st = soax_step(set, layout, integrator, dt, 0, params, nullptr);
  if (st) return st;
  if (nsteps < 0) return fail(SOAX_E_ARG, "nsteps is negative");
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = soax_step(set, layout, integrator, dt, nsteps, params, cap);
    e = hipStreamEndCapture(cap, &g);
  }
  hipGraphExec_t ex = nullptr;
  if (st == SOAX_OK && e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (st) return st;
  if (e != hipSuccess) return hip_fail(e, "step graph capture");
  soax_step_graph* sg = new soax_step_graph();
  sg->set = set;
  sg->generation = set->generation;
  sg->exec = ex;
  *out = sg;
  return SOAX_OK;
}

soax_status soax_step_graph_launch(soax_step_graph* g, void* stream) {
  if (!g) return fail(SOAX_E_ARG, "graph is NULL");
  if (g->set->generation != g->generation)
    return fail(SOAX_E_STATE, "the set changed size or buffers since the steps were captured");
  HIP_TRY(hipGraphLaunch(g->exec, as_stream(stream)), "hipGraphLaunch");
  return SOAX_OK;
}

void soax_step_graph_destroy(soax_step_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  delete g;
}

soax_status soax_aosoa_layout(const soax_schema* schema, int64_t* array_offsets,
                              int64_t* tile_bytes) {
  Layout L;
  soax_status st = parse_schema(schema, L);
  if (st) return st;
  std::vector<int32_t> off;
  const int64_t tb = aosoa_tile(L, &off);
  if (array_offsets)
    for (int a = 0; a < L.narrays; ++a) array_offsets[a] = off[a];
  if (tile_bytes) *tile_bytes = tb;
  return SOAX_OK;
}

soax_status soax_bind_aosoa(soax_set* set, void* aosoa, int64_t bytes) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (!aosoa) {  // detach
    set->aosoa = nullptr;
    set->aosoa_bytes = 0;
    return SOAX_OK;
  }
  const int64_t need = aosoa_need(set->L, set->cap);
  if (bytes < need)
    return fail(SOAX_E_ARG, "the AoSoA buffer holds %lld bytes; %lld are needed for %lld particles",
                static_cast<long long>(bytes), static_cast<long long>(need),
                static_cast<long long>(set->cap));
  if (!aligned16(aosoa)) return fail(SOAX_E_LAYOUT, "the AoSoA buffer is not 16-byte aligned");
  if (!has_soa(set)) return fail(SOAX_E_LAYOUT, "an AoSoA copy needs the SoA copy beside it");
  std::vector<int32_t> off;
  XposeArgs& t = set->aosoa_host;
  t = XposeArgs{};
  t.aos = static_cast<char*>(aosoa);
  t.n = set->n;
  t.stride = static_cast<int32_t>(aosoa_tile(set->L, &off));
  t.narrays = set->L.narrays;
  t.aligned = 1;
  for (const Field& f : set->L.f)
    for (int c = 0; c < f.dim; ++c) {
      const int a = f.first_array + c;
      t.soa[a] = static_cast<char*>(set->soa[a]);
      t.off[a] = off[a];
      t.es[a] = f.es;
    }
  if (!set->aosoa_dev) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(XposeArgs));
    if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(AoSoA table): %s", hipGetErrorString(e));
    set->aosoa_dev = static_cast<XposeArgs*>(d);
  }
  HIP_TRY(hipMemcpy(set->aosoa_dev, &t, sizeof(XposeArgs), hipMemcpyHostToDevice),
          "hipMemcpy(AoSoA table)");
  set->aosoa = static_cast<char*>(aosoa);
  set->aosoa_bytes = bytes;
  return SOAX_OK;
}

static soax_status aosoa_xpose(soax_set* set, bool to_soa, void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (!set->aosoa) return fail(SOAX_E_LAYOUT, "the set has no AoSoA copy");
  if (set->n == 0) return SOAX_OK;
  XposeArgs h = set->aosoa_host;
  h.n = set->n;
  HIP_TRY(launch_aosoa_xpose(to_soa, h, set->aosoa_dev, as_stream(stream)), "AoSoA conversion launch");
  return SOAX_OK;
}

soax_status soax_aosoa_to_soa(soax_set* set, void* stream) { return aosoa_xpose(set, true, stream); }
soax_status soax_soa_to_aosoa(soax_set* set, void* stream) { return aosoa_xpose(set, false, stream); }

soax_status soax_get_record(const soax_set* set, int32_t layout, int64_t i, void* host_record) {
  if (!set || !host_record) return fail(SOAX_E_ARG, "set or host_record is NULL");
  if (i < 0 || i >= set->n) return fail(SOAX_E_ARG, "record %lld out of range", static_cast<long long>(i));
  const Layout& L = set->L;
  char* out = static_cast<char*>(host_record);
  if (layout == SOAX_AOS) {
    if (!has_aos(set)) return fail(SOAX_E_LAYOUT, "the set has no AoS copy");
    HIP_TRY(hipMemcpy(out, set->aos + i * L.stride, L.stride, hipMemcpyDeviceToHost), "hipMemcpy");
    return SOAX_OK;
  }
  if (layout == SOAX_AOSOA) {
    if (!set->aosoa) return fail(SOAX_E_LAYOUT, "the set has no AoSoA copy");
    std::vector<int32_t> off;
    const int64_t tb = aosoa_tile(L, &off);
    memset(out, 0, L.stride);
    const char* tile = set->aosoa + (i / kAosoaW) * tb;
    for (const Field& f : L.f)
      for (int c = 0; c < f.dim; ++c)
        HIP_TRY(hipMemcpy(out + f.off + c * f.es, tile + off[f.first_array + c] + (i % kAosoaW) * f.es,
                          f.es, hipMemcpyDeviceToHost),
                "hipMemcpy");
    return SOAX_OK;
  }
  if (layout != SOAX_SOA) return fail(SOAX_E_ARG, "layout must be SOAX_SOA, SOAX_AOS or SOAX_AOSOA");
  if (set->soa.empty()) return fail(SOAX_E_LAYOUT, "the set has no SoA copy");
  memset(out, 0, L.stride);
  for (const Field& f : L.f)
    for (int c = 0; c < f.dim; ++c)
      HIP_TRY(hipMemcpy(out + f.off + c * f.es,
                        static_cast<const char*>(set->soa[f.first_array + c]) + i * f.es, f.es,
                        hipMemcpyDeviceToHost),
              "hipMemcpy");
  return SOAX_OK;
}

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

// ----------------------------------------------------------- expressions

namespace {

bool valid_dtype(int32_t t) { return t >= kI8 && t <= kF64; }

// Checks a postfix program against `nsrc` available arrays and copies it into
// the plan.
soax_status check_program(const soax_expr_op* prog, int32_t nops, int32_t nsrc, ExprPlan* plan) {
  if (!prog) return fail(SOAX_E_ARG, "prog is NULL");
  if (nops < 1 || nops > kExprMaxOps)
    return fail(SOAX_E_ARG, "nops = %d outside 1..%d", nops, kExprMaxOps);
  int depth = 0, nconst = 0;
  for (int k = 0; k < nops; ++k) {
    const soax_expr_op& o = prog[k];
    switch (o.op) {
      case SOAX_OP_ARRAY:
        if (o.arg < 0 || o.arg >= nsrc) return fail(SOAX_E_ARG, "op %d: array %d out of range", k, o.arg);
        ++depth;
        break;
      case SOAX_OP_CONST:
        if (++nconst > kExprMaxConst) return fail(SOAX_E_ARG, "more than %d constants", kExprMaxConst);
        ++depth;
        break;
      case SOAX_OP_NEG: case SOAX_OP_ABS: case SOAX_OP_SQRT:
        if (depth < 1) return fail(SOAX_E_ARG, "op %d: no operand", k);
        break;
      case SOAX_OP_ADD: case SOAX_OP_SUB: case SOAX_OP_MUL: case SOAX_OP_DIV: case SOAX_OP_MIN:
      case SOAX_OP_MAX:
        if (depth < 2) return fail(SOAX_E_ARG, "op %d: fewer than two operands", k);
        --depth;
        break;
      default:
        return fail(SOAX_E_ARG, "op %d: unknown code %d", k, o.op);
    }
    plan->ops[k] = ExprOp{o.op, o.arg, o.value};
  }
  if (depth != 1) return fail(SOAX_E_ARG, "the program leaves %d values, not 1", depth);
  plan->nops = nops;
  return SOAX_OK;
}

soax_status run_plan(ExprPlan& plan, hipStream_t s) {
  int64_t bytes = dtype_size(plan.dst_t);
  for (int j = 0; j < plan.nsrc; ++j) bytes += dtype_size(plan.src_t[j]);
  plan.stream = plan.n * bytes >= kStreamBytes;
  std::string log;
  const hipError_t e = launch_expr(plan, s, &log);
  if (e != hipSuccess)
    return fail(SOAX_E_HIP, "expression kernel: %s (%s)", hipGetErrorString(e), log.c_str());
  return SOAX_OK;
}

}  // namespace

soax_status soax_eval_ptrs(int64_t n, void* dst, int32_t dst_dtype, const void* const* src,
                           const int32_t* src_dtypes, int32_t nsrc, const soax_expr_op* prog,
                           int32_t nops, void* stream) {
  if (n < 0) return fail(SOAX_E_ARG, "n is negative");
  if (dst_dtype != kF32 && dst_dtype != kF64) return fail(SOAX_E_SCHEMA, "the destination must be f32 or f64");
  if (nsrc < 0 || nsrc > kExprMaxSrc) return fail(SOAX_E_ARG, "nsrc = %d outside 0..%d", nsrc, kExprMaxSrc);
  if (nsrc > 0 && (!src || !src_dtypes)) return fail(SOAX_E_ARG, "src or src_dtypes is NULL");
  if (n > 0 && !dst) return fail(SOAX_E_ARG, "dst is NULL");
  ExprPlan plan{};
  for (int j = 0; j < nsrc; ++j) {
    if (!valid_dtype(src_dtypes[j])) return fail(SOAX_E_SCHEMA, "src_dtypes[%d] = %d is unknown", j, src_dtypes[j]);
    if (n > 0 && !src[j]) return fail(SOAX_E_ARG, "src[%d] is NULL", j);
    plan.src[j] = src[j];
    plan.src_t[j] = src_dtypes[j];
  }
  soax_status st;
  if ((st = check_program(prog, nops, nsrc, &plan))) return st;
  plan.nsrc = nsrc;
  plan.dst = dst;
  plan.dst_t = dst_dtype;
  plan.n = n;
  return run_plan(plan, as_stream(stream));
}

soax_status soax_eval(soax_set* set, int32_t dst_array, const soax_expr_op* prog, int32_t nops,
                      void* stream) {
  if (!set) return fail(SOAX_E_ARG, "set is NULL");
  if (!has_soa(set)) return fail(SOAX_E_LAYOUT, "the set has no SoA copy");
  const Layout& L = set->L;
  if (dst_array < 0 || dst_array >= L.narrays)
    return fail(SOAX_E_ARG, "dst_array %d out of range", dst_array);
  std::vector<int32_t> type_of(L.narrays);
  for (const Field& f : L.f)
    for (int c = 0; c < f.dim; ++c) type_of[f.first_array + c] = f.dtype;
  if (type_of[dst_array] != kF32 && type_of[dst_array] != kF64)
    return fail(SOAX_E_SCHEMA, "the destination array must be f32 or f64");
  // the set's arrays the program reads, renumbered 0.. in order of first use
  if (!prog) return fail(SOAX_E_ARG, "prog is NULL");
  if (nops < 1 || nops > kExprMaxOps) return fail(SOAX_E_ARG, "nops = %d outside 1..%d", nops, kExprMaxOps);
  std::vector<soax_expr_op> local(prog, prog + nops);
  std::vector<int> slot(L.narrays, -1);
  ExprPlan plan{};
  int nsrc = 0;
  for (soax_expr_op& o : local) {
    if (o.op != SOAX_OP_ARRAY) continue;
    if (o.arg < 0 || o.arg >= L.narrays) return fail(SOAX_E_ARG, "array %d out of range", o.arg);
    if (slot[o.arg] < 0) {
      if (nsrc == kExprMaxSrc) return fail(SOAX_E_ARG, "more than %d distinct arrays", kExprMaxSrc);
      slot[o.arg] = nsrc;
      plan.src[nsrc] = set->soa[o.arg];
      plan.src_t[nsrc] = type_of[o.arg];
      ++nsrc;
    }
    o.arg = slot[o.arg];
  }
  soax_status st;
  if ((st = check_program(local.data(), nops, nsrc, &plan))) return st;
  plan.nsrc = nsrc;
  plan.dst = set->soa[dst_array];
  plan.dst_t = type_of[dst_array];
  plan.n = set->n;
  return run_plan(plan, as_stream(stream));
}

soax_status soax_expr_source(const soax_expr_op* prog, int32_t nops, int32_t dst_dtype,
                             const int32_t* src_dtypes, int32_t nsrc, char* buf, int64_t size) {
  if (dst_dtype != kF32 && dst_dtype != kF64) return fail(SOAX_E_SCHEMA, "the destination must be f32 or f64");
  if (nsrc < 0 || nsrc > kExprMaxSrc) return fail(SOAX_E_ARG, "nsrc = %d outside 0..%d", nsrc, kExprMaxSrc);
  if (nsrc > 0 && !src_dtypes) return fail(SOAX_E_ARG, "src_dtypes is NULL");
  if (!buf || size < 1) return fail(SOAX_E_ARG, "buf is NULL or empty");
  ExprPlan plan{};
  for (int j = 0; j < nsrc; ++j) {
    if (!valid_dtype(src_dtypes[j])) return fail(SOAX_E_SCHEMA, "src_dtypes[%d] = %d is unknown", j, src_dtypes[j]);
    plan.src_t[j] = src_dtypes[j];
  }
  soax_status st;
  if ((st = check_program(prog, nops, nsrc, &plan))) return st;
  plan.nsrc = nsrc;
  plan.dst_t = dst_dtype;
  const std::string src = expr_source(plan);
  if (static_cast<int64_t>(src.size()) + 1 > size)
    return fail(SOAX_E_ARG, "buf holds %lld bytes; the source needs %zu", static_cast<long long>(size),
                src.size() + 1);
  memcpy(buf, src.c_str(), src.size() + 1);
  return SOAX_OK;
}

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

// --------------------------------------------------------------- batching

}  // extern "C"

namespace {

void drop_graphs(soax_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// (Re)build the tile list for the current tile size and upload it together
// with the set table (whose tile offsets depend on it).  Drains the device
// first: a replaced list may still be read by work in flight.
soax_status build_tiles(soax_batch* b) {
  const int tile = b->block * b->per_thread;
  if (b->tile_for == tile) return SOAX_OK;
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  b->stage_pending = false;
  std::vector<int32_t> tile_set;
  for (size_t si = 0; si < b->sets.size(); ++si) {
    b->stage[si].tile_begin = static_cast<int64_t>(tile_set.size());
    const int64_t nt = (b->sets[si]->n + tile - 1) / tile;
    for (int64_t t = 0; t < nt; ++t) tile_set.push_back(static_cast<int32_t>(si));
  }
  if (tile_set.size() > static_cast<size_t>(INT32_MAX))
    return fail(SOAX_E_RANGE, "too many tiles");
  if (b->dev_tile_set) {
    (void)hipFree(b->dev_tile_set);
    b->dev_tile_set = nullptr;
  }
  b->ntiles = static_cast<int64_t>(tile_set.size());
  if (b->ntiles > 0) {
    hipError_t e = hipMalloc(&b->dev_tile_set, tile_set.size() * sizeof(int32_t));
    if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(tile list): %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpy(b->dev_tile_set, tile_set.data(), tile_set.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice),
            "hipMemcpy(tile list)");
  }
  HIP_TRY(hipMemcpy(b->dev_sets, b->stage, b->sets.size() * sizeof(BatchSet), hipMemcpyHostToDevice),
          "hipMemcpy(set table)");
  b->tile_for = tile;
  drop_graphs(b);
  return SOAX_OK;
}

BatchLaunch batch_launch(const soax_batch* b) {
  BatchLaunch L{};
  L.sets = b->dev_sets;
  L.tile_set = b->dev_tile_set;
  L.ntiles = b->ntiles;
  L.nsets = static_cast<int32_t>(b->sets.size());
  L.tile = b->block * b->per_thread;
  L.block = b->block;
  L.per_thread = b->per_thread;
  int64_t grid = static_cast<int64_t>(b->cus) * b->blocks_per_cu;
  if (grid > b->ntiles) grid = b->ntiles;
  L.grid = static_cast<int32_t>(std::max<int64_t>(grid, 1));
  L.vel_t = b->vel_t;
  return L;
}

// Copy dt/abc into the pinned staging table and enqueue its upload.
soax_status upload_params(soax_batch* b, const double* dt, const double* abc, hipStream_t s) {
  if (b->stage_pending) {
    HIP_TRY(hipEventSynchronize(b->stage_done), "hipEventSynchronize");
    b->stage_pending = false;
  }
  for (size_t i = 0; i < b->sets.size(); ++i) {
    b->stage[i].small = small_steps(dt[i], abc[3 * i], abc[3 * i + 1], abc[3 * i + 2]) ? 1 : 0;
    b->stage[i].dt = dt[i];
    b->stage[i].A = abc[3 * i];
    b->stage[i].B = abc[3 * i + 1];
    b->stage[i].C = abc[3 * i + 2];
  }
  HIP_TRY(hipMemcpyAsync(b->dev_sets, b->stage, b->sets.size() * sizeof(BatchSet),
                         hipMemcpyHostToDevice, s),
          "hipMemcpyAsync(set table)");
  HIP_TRY(hipEventRecord(b->stage_done, s), "hipEventRecord");
  b->stage_pending = true;
  return SOAX_OK;
}

// A set resized or regrown since the batch was made invalidates the batch's
// tables (sizes, pointers, tiles, captured graphs).
soax_status check_generations(const soax_batch* b) {
  for (size_t i = 0; i < b->sets.size(); ++i)
    if (b->sets[i]->generation != b->generations[i])
      return fail(SOAX_E_STATE, "set %zu changed size since the batch was created", i);
  return SOAX_OK;
}

soax_status per_set_step(soax_batch* b, const double* dt, const double* abc, hipStream_t s) {
  for (size_t i = 0; i < b->sets.size(); ++i) {
    soax_set* set = b->sets[i];
    const Layout& L = set->L;
    const int fp = L.find("pos"), fv = L.find("vel");
    SoaStepArgs a{};
    for (int d = 0; d < 3; ++d) {
      a.pos[d] = set->soa[L.f[fp].first_array + d];
      a.vel[d] = set->soa[L.f[fv].first_array + d];
    }
    a.n = set->n;
    a.dt = dt[i];
    a.abc = AbcParams{abc[3 * i], abc[3 * i + 1], abc[3 * i + 2]};
    a.wrap = 1;
    HIP_TRY(launch_soa_step(kRk2Abc, kF64, b->vel_t, 1, 128, a, s), "per-set step launch");
  }
  return SOAX_OK;
}

soax_status graph_for(soax_batch* b, int64_t nsteps, hipGraphExec_t* out) {
  auto key = std::make_tuple(nsteps, b->block, b->per_thread, b->blocks_per_cu);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return SOAX_OK;
  }
  const BatchLaunch L = batch_launch(b);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal),
          "hipStreamBeginCapture");
  hipError_t e = hipSuccess;
  for (int64_t k = 0; k < nsteps && e == hipSuccess; ++k) e = launch_batch_rk2(L, b->capture_stream);
  hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "captured batch launch");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (b->graphs.size() >= 8) drop_graphs(b);
  b->graphs[key] = ex;
  *out = ex;
  return SOAX_OK;
}

}  // namespace

extern "C" {

soax_status soax_batch_create(soax_set* const* sets, int32_t nsets, soax_batch** out) {
  if (!out) return fail(SOAX_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sets || nsets < 1) return fail(SOAX_E_ARG, "need at least one set");
  int vel_t = 0;
  int64_t total = 0;
  for (int i = 0; i < nsets; ++i) {
    soax_set* s = sets[i];
    if (!s) return fail(SOAX_E_ARG, "sets[%d] is NULL", i);
    int fp, fv;
    soax_status st;
    if ((st = vec_field(s->L, "pos", &fp)) || (st = vec_field(s->L, "vel", &fv))) return st;
    if (s->L.f[fp].dtype != kF64) return fail(SOAX_E_SCHEMA, "batched RK2 needs f64 'pos'");
    if (i == 0) vel_t = s->L.f[fv].dtype;
    if (s->L.f[fv].dtype != vel_t) return fail(SOAX_E_SCHEMA, "every set needs the same 'vel' type");
    if (s->soa.empty() && s->n > 0) return fail(SOAX_E_LAYOUT, "sets[%d] has no SoA copy", i);
    if (s->n > 0 && !s->soa_vec_ok) return fail(SOAX_E_LAYOUT, "sets[%d] arrays are not 16-byte aligned", i);
    total += s->n;
  }
  soax_batch* b = new soax_batch();
  b->sets.assign(sets, sets + nsets);
  for (int i = 0; i < nsets; ++i) b->generations.push_back(sets[i]->generation);
  b->vel_t = vel_t;
  b->total = total;
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  b->cus = prop.multiProcessorCount;
  b->arch = prop.gcnArchName;
  soax_status st = SOAX_OK;
  e = hipHostMalloc(reinterpret_cast<void**>(&b->stage), nsets * sizeof(BatchSet), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&b->dev_sets, nsets * sizeof(BatchSet));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) st = hip_fail(e, "batch set-up");
  if (st == SOAX_OK) {
    for (int i = 0; i < nsets; ++i) {
      soax_set* s = sets[i];
      const int fp = s->L.find("pos"), fv = s->L.find("vel");
      BatchSet& t = b->stage[i];
      memset(&t, 0, sizeof t);
      for (int d = 0; d < 3; ++d) {
        t.pos[d] = s->n ? static_cast<double*>(s->soa[s->L.f[fp].first_array + d]) : nullptr;
        t.vel[d] = s->n ? s->soa[s->L.f[fv].first_array + d] : nullptr;
      }
      t.n = s->n;
    }
    st = build_tiles(b);
  }
  if (st != SOAX_OK) {
    soax_batch_destroy(b);
    return st;
  }
  *out = b;
  return SOAX_OK;
}

void soax_batch_destroy(soax_batch* b) {
  if (!b) return;
  if (b->stage_pending) (void)hipEventSynchronize(b->stage_done);
  drop_graphs(b);
  if (b->dev_tile_set) (void)hipFree(b->dev_tile_set);
  if (b->dev_sets) (void)hipFree(b->dev_sets);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->stage_done) (void)hipEventDestroy(b->stage_done);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
}

soax_status soax_batch_config(soax_batch* b, int32_t block, int32_t per_thread, int32_t blocks_per_cu) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (block != 0 && (block < 64 || block > 512 || block % 64))
    return fail(SOAX_E_ARG, "block %d must be 0 or a multiple of 64 in 64..512", block);
  if (per_thread != 0 && per_thread != 1 && per_thread != 2 && per_thread != 4)
    return fail(SOAX_E_ARG, "per_thread %d must be 0, 1, 2 or 4", per_thread);
  if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(SOAX_E_ARG, "blocks_per_cu must be 0..64");
  if (block) b->block = block;
  if (per_thread) b->per_thread = per_thread;
  if (blocks_per_cu) b->blocks_per_cu = blocks_per_cu;
  drop_graphs(b);
  return build_tiles(b);
}

soax_status soax_batch_get_config(const soax_batch* b, int32_t* block, int32_t* per_thread,
                                  int32_t* blocks_per_cu) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (block) *block = b->block;
  if (per_thread) *per_thread = b->per_thread;
  if (blocks_per_cu) *blocks_per_cu = b->blocks_per_cu;
  return SOAX_OK;
}

soax_status soax_batch_step(soax_batch* b, const double* dt, const double* abc, int64_t nsteps,
                            int32_t mode, void* stream) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  if (!dt || !abc) return fail(SOAX_E_ARG, "dt or abc is NULL");
  if (nsteps < 0) return fail(SOAX_E_ARG, "nsteps is negative");
  if (mode < 0 || mode > 2) return fail(SOAX_E_ARG, "mode must be 0, 1 or 2");
  soax_status st0 = check_generations(b);
  if (st0) return st0;
  for (size_t i = 0; i < b->sets.size(); ++i) {
    if (!is_finite(dt[i])) return fail(SOAX_E_ARG, "dt[%zu] is not finite", i);
    for (int j = 0; j < 3; ++j)
      if (!is_finite(abc[3 * i + j])) return fail(SOAX_E_ARG, "abc[%zu] is not finite", 3 * i + j);
  }
  hipStream_t s = as_stream(stream);
  if (nsteps == 0) return SOAX_OK;
  if (mode == 0) {
    for (int64_t k = 0; k < nsteps; ++k) {
      soax_status st = per_set_step(b, dt, abc, s);
      if (st) return st;
    }
    return SOAX_OK;
  }
  soax_status st = upload_params(b, dt, abc, s);
  if (st) return st;
  if (mode == 1) {
    const BatchLaunch L = batch_launch(b);
    for (int64_t k = 0; k < nsteps; ++k) HIP_TRY(launch_batch_rk2(L, s), "batch launch");
    return SOAX_OK;
  }
  hipGraphExec_t ex = nullptr;
  if ((st = graph_for(b, nsteps, &ex))) return st;
  HIP_TRY(hipGraphLaunch(ex, s), "hipGraphLaunch");
  return SOAX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuner

namespace {

struct TuneEntry {
  int block, per_thread, blocks_per_cu;
  double ms;
};

// The cache is a JSON object with one entry per line:
//   "key": {"block": B, "per_thread": P, "blocks_per_cu": C, "ms": T},
std::map<std::string, TuneEntry> read_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char key[512];
    TuneEntry e{};
    if (sscanf(line, " \"%511[^\"]\": {\"block\": %d, \"per_thread\": %d, \"blocks_per_cu\": %d, \"ms\": %lf",
               key, &e.block, &e.per_thread, &e.blocks_per_cu, &e.ms) == 5)
      m[key] = e;
  }
  fclose(f);
  return m;
}

bool write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f, "\"%s\": {\"block\": %d, \"per_thread\": %d, \"blocks_per_cu\": %d, \"ms\": %.6f}%s\n",
            kv.first.c_str(), kv.second.block, kv.second.per_thread, kv.second.blocks_per_cu,
            kv.second.ms, (++i < m.size()) ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  return rename(tmp.c_str(), path) == 0;
}

// Device copies of every set's pos and vel, to restore them after timing.
struct Snapshot {
  std::vector<void*> bufs;
  ~Snapshot() {
    for (void* p : bufs) (void)hipFree(p);
  }
};

soax_status snapshot(soax_batch* b, Snapshot& snap, bool restore) {
  size_t k = 0;
  for (soax_set* s : b->sets) {
    if (s->n == 0) continue;
    const int fp = s->L.find("pos"), fv = s->L.find("vel");
    for (int d = 0; d < 3; ++d) {
      for (int which = 0; which < 2; ++which) {
        const Field& f = s->L.f[which ? fv : fp];
        void* arr = s->soa[f.first_array + d];
        const size_t bytes = static_cast<size_t>(s->n) * f.es;
        if (!restore) {
          void* p = nullptr;
          hipError_t e = hipMalloc(&p, bytes);
          if (e != hipSuccess) return fail(SOAX_E_OOM, "hipMalloc(tuning snapshot): %s", hipGetErrorString(e));
          snap.bufs.push_back(p);
          HIP_TRY(hipMemcpy(p, arr, bytes, hipMemcpyDeviceToDevice), "hipMemcpy(snapshot)");
        } else {
          HIP_TRY(hipMemcpy(arr, snap.bufs[k++], bytes, hipMemcpyDeviceToDevice), "hipMemcpy(restore)");
        }
      }
    }
  }
  return SOAX_OK;
}

}  // namespace

extern "C" soax_status soax_batch_tune(soax_batch* b, const char* cache_path) {
  if (!b) return fail(SOAX_E_ARG, "batch is NULL");
  soax_status st0 = check_generations(b);
  if (st0) return st0;
  char keybuf[256];
  snprintf(keybuf, sizeof keybuf, "%s|batch_rk2|vel%d|sets=%zu|n=%lld", b->arch.c_str(), b->vel_t,
           b->sets.size(), static_cast<long long>(b->total));
  const std::string key = keybuf;
  std::map<std::string, TuneEntry> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end())
      return soax_batch_config(b, it->second.block, it->second.per_thread, it->second.blocks_per_cu);
  }
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  Snapshot snap;
  soax_status st = snapshot(b, snap, false);
  if (st) return st;
  // timing runs use the amplitudes and dt already in the device table
  std::vector<double> dts(b->sets.size(), 1e-3), abc(3 * b->sets.size(), 1.0);
  if ((st = upload_params(b, dts.data(), abc.data(), nullptr))) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  const int blocks[] = {128, 256, 512};
  const int ppts[] = {1, 2, 4};
  const int bpcs[] = {2, 4, 8, 16, 32, 64};
  TuneEntry best{b->block, b->per_thread, b->blocks_per_cu, 1e30};
  for (int bl : blocks)
    for (int pp : ppts)
      for (int bc : bpcs) {
        if ((st = soax_batch_config(b, bl, pp, bc))) break;
        const BatchLaunch L = batch_launch(b);
        hipError_t e = launch_batch_rk2(L, nullptr);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_batch_rk2(L, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = hip_fail(e, "tuning run");
          break;
        }
        if (ms / 3 < best.ms) best = TuneEntry{bl, pp, bc, ms / 3.0};
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  soax_status rst = snapshot(b, snap, true);
  if (st) return st;
  if (rst) return rst;
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if ((st = soax_batch_config(b, best.block, best.per_thread, best.blocks_per_cu))) return st;
  if (cache_path) {
    cache[key] = best;
    if (!write_cache(cache_path, cache)) return fail(SOAX_E_ARG, "cannot write tuning cache '%s'", cache_path);
  }
  return SOAX_OK;
}

// --------------------------------------------------------------- utilities

extern "C" soax_status soax_copy(void* dst, const void* src, int64_t bytes, void* stream) {
  if ((!dst || !src) && bytes > 0) return fail(SOAX_E_ARG, "dst or src is NULL");
  if (bytes < 0) return fail(SOAX_E_ARG, "bytes is negative");
  if (!aligned16(dst) || !aligned16(src)) return fail(SOAX_E_ARG, "copy needs 16-byte aligned pointers");
  if (bytes == 0) return SOAX_OK;
  HIP_TRY(launch_copy16(dst, src, bytes, as_stream(stream)), "copy launch");
  return SOAX_OK;
}

extern "C" const char* soax_strerror(soax_status st) {
  switch (st) {
    case SOAX_OK: return "ok";
    case SOAX_E_ARG: return "invalid argument";
    case SOAX_E_SCHEMA: return "invalid schema";
    case SOAX_E_RANGE: return "size out of range";
    case SOAX_E_LAYOUT: return "layout unavailable";
    case SOAX_E_OOM: return "out of device memory";
    case SOAX_E_HIP: return "HIP runtime error";
    case SOAX_E_STATE: return "invalid state";
    default: return "unknown status";
  }
}

extern "C" const char* soax_last_error(void) { return g_last_error.c_str(); }
