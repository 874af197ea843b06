// soax_host.cpp -- host side of the C ABI (include/soax.h) for particle
// sets: creation and binding, fill, steps in every layout, transposes,
// captured step graphs, the AoSoA copy, records, and the utilities.  Every
// argument is checked before any device call.
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

struct soax_step_graph {
  soax_set* set = nullptr;
  uint64_t generation = 0;  // of the set when captured
  hipGraphExec_t exec = nullptr;
};

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
    // one particle per thread in workgroups of 128, except, for the field
    // integrators on sets that stream through HBM, two consecutive particles
    // (16-byte position accesses) in workgroups of 64: the fastest shapes
    // measured on the MI355X at 1e8 particles (two per thread: RK2 and Heun
    // 3% faster than one, RK4 2%, Euler 10% slower; then 64 threads: RK2 and
    // Heun about 1% faster than 128 in interleaved runs, RK4 level, Euler 6%
    // slower).  Cache-resident sets are bound by latency, and there the wider
    // shape was slower (one launch per set over 256 sets of 1e3..1e6
    // particles: 174 ms against 150 ms for 100 steps).
    const bool wide = field_integrator(integrator) &&
                      set->n * soa_step_bytes(integrator, L.f[fp].es, L.f[fv].es) >= kStreamBytes;
    int vec = set->vec ? set->vec : (wide ? 2 : 1);
    if (!set->soa_vec_ok) vec = 1;
    // four particles per thread would split each 8-byte array's 32-byte run
    // into two 16-byte accesses, each covering every other half of the wave's
    // lines: measured 3x slower at 1e8, so 8-byte positions or velocities
    // take at most two
    if (vec > 2 && (L.f[fp].es == 8 || L.f[fv].es == 8)) vec = 2;
    const int block = set->block[SOAX_SOA] ? set->block[SOAX_SOA] : (wide ? 64 : 128);
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

soax_status soax_step_fused(soax_set* set, int32_t integrator, double dt, int64_t nsteps,
                            const soax_params* params, void* stream) {
  // every argument check of soax_step on the SoA arrays, with nothing launched
  soax_status st = soax_step(set, SOAX_SOA, integrator, dt, 0, params, nullptr);
  if (st) return st;
  if (nsteps < 0) return fail(SOAX_E_ARG, "nsteps is negative");
  const Layout& L = set->L;
  int fp, fv, fa = -1;
  (void)vec_field(L, "pos", &fp);
  (void)vec_field(L, "vel", &fv);
  if (uses_acc(integrator)) (void)vec_field(L, "acc", &fa);
  SoaStepArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.pos[d] = set->soa[L.f[fp].first_array + d];
    a.vel[d] = set->soa[L.f[fv].first_array + d];
    a.acc[d] = fa >= 0 ? set->soa[L.f[fa].first_array + d] : nullptr;
  }
  a.n = set->n;
  a.dt = dt;
  if (params) a.abc = AbcParams{params->A, params->B, params->C};
  a.wrap = params ? params->wrap : 0;
  // one particle per thread: the loop over steps is bound by arithmetic, and
  // the arrays are touched once per call
  HIP_TRY(launch_soa_fused(integrator, L.f[fp].dtype, L.f[fv].dtype, 256, a, nsteps,
                           as_stream(stream)),
          "fused SoA step launch");
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
  group_by_size(t);
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

}  // extern "C"

// --------------------------------------------------------------- utilities

extern "C" soax_status soax_copy(void* dst, const void* src, int64_t bytes, void* stream) {
  if ((!dst || !src) && bytes > 0) return fail(SOAX_E_ARG, "dst or src is NULL");
  if (bytes < 0) return fail(SOAX_E_ARG, "bytes is negative");
  if (!aligned16(dst) || !aligned16(src)) return fail(SOAX_E_ARG, "copy needs 16-byte aligned pointers");
  if (bytes == 0) return SOAX_OK;
  HIP_TRY(launch_copy16(dst, src, bytes, as_stream(stream)), "copy launch");
  return SOAX_OK;
}

extern "C" soax_status soax_probe(int32_t pattern, double* const* pos, float* const* vel,
                                  int64_t n, void* stream) {
  if (pattern < kProbeRk2 || pattern > kProbeWrite) return fail(SOAX_E_ARG, "unknown probe pattern %d", pattern);
  if (n < 0 || n > kMaxParticles) return fail(n < 0 ? SOAX_E_ARG : SOAX_E_RANGE, "bad n");
  if (n == 0) return SOAX_OK;
  if (!pos || !pos[0] || !pos[1] || !pos[2]) return fail(SOAX_E_ARG, "pos is NULL");
  const bool writes_vel = pattern == kProbeRk2 || pattern == kProbeEuler || pattern == kProbeWrite;
  if (writes_vel && (!vel || !vel[0] || !vel[1] || !vel[2])) return fail(SOAX_E_ARG, "vel is NULL");
  ProbeArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.pos[d] = pos[d];
    a.vel[d] = writes_vel ? vel[d] : nullptr;
  }
  a.n = n;
  a.c = pattern == kProbeRead ? __builtin_nan("") : 0.0;
  HIP_TRY(launch_stream_probe(pattern, a, as_stream(stream)), "probe launch");
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

extern "C" const char* soax_last_error(void) { return last_error(); }
