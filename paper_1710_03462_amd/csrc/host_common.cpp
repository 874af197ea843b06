// host_common.cpp -- error reporting, schema parsing and the particle-set
// buffer helpers shared by the host side of the C ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "host_internal.h"

namespace soax {
namespace host {

namespace {
thread_local std::string g_last_error;
}  // namespace

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

const char* last_error() { return g_last_error.c_str(); }

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

// A 3-vector float property, or -1 with an error recorded.
soax_status vec_field(const Layout& L, const char* name, int* idx) {
  const int f = L.find(name);
  if (f < 0) return fail(SOAX_E_SCHEMA, "schema has no '%s' property", name);
  if (L.f[f].dim != 3 || !is_real(L.f[f].dtype))
    return fail(SOAX_E_SCHEMA, "'%s' must be a 3-component f32/f64 property", name);
  *idx = f;
  return SOAX_OK;
}

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
  group_by_size(t);
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

}  // namespace host
}  // namespace soax
