// host_expr.cpp -- host side of the fused array expressions: program
// checks and the plan handed to the run-time kernel generator.
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

extern "C" {

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

}  // extern "C"
