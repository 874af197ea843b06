// expr.cpp -- fused element-wise expressions over particle arrays.
//
// Whole-array expressions such as pos_0 = vel_1 - vel_2 (the array access
// and expression templates of Section 4.1-4.2, which fuse an expression into
// a single loop) are compiled at run time into one gfx950 kernel: the
// postfix program is turned into straight-line HIP source (one load per
// distinct array, one double operation per program step, one store), which
// hipRTC compiles once per program shape and device; constants and array
// pointers travel as kernel arguments, so programs that differ only in them
// share a kernel.  Every operation is an IEEE double operation rounded once
// (no contraction into fused multiply-adds) and the result is rounded once to
// the destination type.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "launch.h"

namespace soax {

namespace {

// Kernel arguments; the generated source declares the same struct.
struct ExprArgs {
  const void* src[kExprMaxSrc];
  void* dst;
  long long n;
  double c[kExprMaxConst];
};

const char* ctype(int32_t t) {
  switch (t) {
    case kI8: return "signed char";
    case kU8: return "unsigned char";
    case kI32: return "int";
    case kI64: return "long long";
    case kF32: return "float";
    default: return "double";
  }
}

// Buffer-load and -store expressions of one element of type t at element
// offset `e` of window `w` (a buffer resource over the workgroup's run of the
// array; see the streaming kernels of the library): nt loads, write-through
// nt stores (sc0 sc1 nt).
const char* win_load(int32_t t) {
  switch (t) {
    case kI8: return "(double)(signed char)__builtin_amdgcn_raw_buffer_load_b8(%s, %s, 0, 2)";
    case kU8: return "(double)__builtin_amdgcn_raw_buffer_load_b8(%s, %s, 0, 2)";
    case kI32: return "(double)(int)__builtin_amdgcn_raw_buffer_load_b32(%s, (%s) * 4, 0, 2)";
    case kI64:
      return "(double)__builtin_bit_cast(long long, __builtin_amdgcn_raw_buffer_load_b64(%s, (%s) * 8, 0, 2))";
    case kF32:
      return "(double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(%s, (%s) * 4, 0, 2))";
    default:
      return "__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(%s, (%s) * 8, 0, 2))";
  }
}

std::string win_store(int32_t t, const std::string& value, const char* w, const char* e) {
  char buf[1024];
  switch (t) {
    case kI8:
    case kU8:
      snprintf(buf, sizeof buf, "  __builtin_amdgcn_raw_buffer_store_b8((unsigned char)(%s)(%s), %s, %s, 0, 19);\n",
               ctype(t), value.c_str(), w, e);
      break;
    case kI32:
      snprintf(buf, sizeof buf, "  __builtin_amdgcn_raw_buffer_store_b32((unsigned)(int)(%s), %s, (%s) * 4, 0, 19);\n",
               value.c_str(), w, e);
      break;
    case kF32:
      snprintf(buf, sizeof buf,
               "  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)(%s)), %s, (%s) * 4, 0, 19);\n",
               value.c_str(), w, e);
      break;
    case kI64:
      snprintf(buf, sizeof buf,
               "  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, (long long)(%s)), %s, (%s) * 8, 0, 19);\n",
               value.c_str(), w, e);
      break;
    default:
      snprintf(buf, sizeof buf,
               "  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, (double)(%s)), %s, (%s) * 8, 0, 19);\n",
               value.c_str(), w, e);
      break;
  }
  return buf;
}

int elem_size(int32_t t) {
  switch (t) {
    case kI8: case kU8: return 1;
    case kI32: case kF32: return 4;
    default: return 8;
  }
}

// Each thread evaluates two elements a block-width apart: both elements'
// loads, then both elements' arithmetic, then both stores.  A thread alone
// reads and writes its two elements, so a destination that is also a source
// is still read before it is written.  Past the end of the array the second
// element is element i0 again (loaded and stored with the first one's value),
// so no load or store sits behind a branch: the compiler would otherwise sink
// the second element's loads below the first element's store.
constexpr int kExprBlock = 256;
constexpr int kExprPerThread = 2;

// Straight-line source of one program; `consts` receives the constant values
// in the order the source refers to them.
std::string generate(const ExprPlan& p, std::vector<double>* consts) {
  std::string s;
  char buf[1024];
  s += "typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));\n";
  s += "struct Args { const void* src[" + std::to_string(kExprMaxSrc) +
       "]; void* dst; long long n; double c[" + std::to_string(kExprMaxConst) + "]; };\n";
  s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(kExprBlock) +
       ") soax_expr_kernel(Args a) {\n";
  s += "  const long long i0 = (long long)blockIdx.x * " + std::to_string(kExprBlock * kExprPerThread) +
       " + threadIdx.x;\n";
  s += "  if (i0 >= a.n) return;\n";
  s += "  const long long i1 = i0 + " + std::to_string(kExprBlock) + ";\n";
  s += "  const bool has1 = i1 < a.n;\n";
  s += "  const long long j1 = has1 ? i1 : i0;\n";
  std::vector<bool> used(kExprMaxSrc, false);
  for (int k = 0; k < p.nops; ++k)
    if (p.ops[k].op == kOpArray) used[p.ops[k].arg] = true;
  if (p.stream) {
    // the workgroup's run of every array, and each element's offset in it
    s += "  const long long first = (long long)blockIdx.x * " +
         std::to_string(kExprBlock * kExprPerThread) + ";\n";
    s += "  const long long cnt = a.n - first < " + std::to_string(kExprBlock * kExprPerThread) +
         " ? a.n - first : " + std::to_string(kExprBlock * kExprPerThread) + ";\n";
    s += "  const int e0 = (int)(i0 - first), e1 = (int)(j1 - first);\n";
    for (int j = 0; j < p.nsrc; ++j) {
      if (!used[j]) continue;
      const int es = elem_size(p.src_t[j]);
      snprintf(buf, sizeof buf,
               "  const __amdgpu_buffer_rsrc_t w%d = __builtin_amdgcn_make_buffer_rsrc("
               "(char*)a.src[%d] + first * %d, 0, (int)(cnt * %d), 0x00020000);\n",
               j, j, es, es);
      s += buf;
    }
    const int es = elem_size(p.dst_t);
    snprintf(buf, sizeof buf,
             "  const __amdgpu_buffer_rsrc_t wd = __builtin_amdgcn_make_buffer_rsrc("
             "(char*)a.dst + first * %d, 0, (int)(cnt * %d), 0x00020000);\n",
             es, es);
    s += buf;
  }
  for (int e = 0; e < kExprPerThread; ++e)
    for (int j = 0; j < p.nsrc; ++j) {
      if (!used[j]) continue;
      const char* t = ctype(p.src_t[j]);
      const char* idx = e == 0 ? "i0" : "j1";
      if (p.stream) {
        char w[8], load[512];
        snprintf(w, sizeof w, "w%d", j);
        snprintf(load, sizeof load, win_load(p.src_t[j]), w, e == 0 ? "e0" : "e1");
        snprintf(buf, sizeof buf, "  const double s%d_%d = %s;\n", j, e, load);
      } else {
        snprintf(buf, sizeof buf, "  const double s%d_%d = (double)((const %s*)a.src[%d])[%s];\n", j, e, t,
                 j, idx);
      }
      s += buf;
    }
  // constant k of the program is a.c[cidx[k]]
  std::vector<int> cidx(p.nops, -1);
  for (int k = 0; k < p.nops; ++k)
    if (p.ops[k].op == kOpConst) {
      cidx[k] = static_cast<int>(consts->size());
      consts->push_back(p.ops[k].value);
    }
  const char* dt = ctype(p.dst_t);
  std::string result[kExprPerThread];
  for (int el = 0; el < kExprPerThread; ++el) {
    const std::string sfx = "_" + std::to_string(el);
    std::vector<std::string> stack;
    for (int k = 0; k < p.nops; ++k) {
      const ExprOp& o = p.ops[k];
      const std::string v = "t" + std::to_string(k) + sfx;
      if (o.op == kOpArray) {
        stack.push_back("s" + std::to_string(o.arg) + sfx);
        continue;
      }
      if (o.op == kOpConst) {
        stack.push_back("a.c[" + std::to_string(cidx[k]) + "]");
        continue;
      }
      std::string e;
      if (o.op == kOpNeg || o.op == kOpAbs || o.op == kOpSqrt) {
        const std::string x = stack.back();
        stack.pop_back();
        if (o.op == kOpNeg) e = "-(" + x + ")";
        else if (o.op == kOpAbs) e = "__builtin_fabs(" + x + ")";
        else e = "__builtin_sqrt(" + x + ")";
      } else {
        const std::string b = stack.back();
        stack.pop_back();
        const std::string a = stack.back();
        stack.pop_back();
        switch (o.op) {
          case kOpAdd: e = a + " + " + b; break;
          case kOpSub: e = a + " - " + b; break;
          case kOpMul: e = a + " * " + b; break;
          case kOpDiv: e = a + " / " + b; break;
          case kOpMin: e = "(" + a + " < " + b + " ? " + a + " : " + b + ")"; break;
          default: e = "(" + a + " > " + b + " ? " + a + " : " + b + ")"; break;
        }
      }
      s += "  const double " + v + " = " + e + ";\n";
      stack.push_back(v);
    }
    result[el] = stack.back();
  }
  const std::string value[kExprPerThread] = {result[0],
                                             "has1 ? " + result[1] + " : " + result[0]};
  for (int el = 0; el < kExprPerThread; ++el) {
    const char* idx = el == 0 ? "i0" : "j1";
    if (p.stream) {
      s += win_store(p.dst_t, value[el], "wd", el == 0 ? "e0" : "e1");
    } else {
      snprintf(buf, sizeof buf, "  ((%s*)a.dst)[%s] = (%s)(%s);\n", dt, idx, dt, value[el].c_str());
      s += buf;
    }
  }
  s += "}\n";
  return s;
}

struct Compiled {
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
};

std::mutex g_mu;
std::map<std::tuple<int, std::string>, Compiled> g_cache;

hipError_t compile(const std::string& src, const std::string& arch, Compiled* out, std::string* log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "soax_expr.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return hipErrorInvalidValue;
  }
  const std::string arch_opt = "--offload-arch=" + arch;
  const char* opts[] = {arch_opt.c_str(), "-O3", "-ffp-contract=off", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string l(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &l[0]);
    *log = std::string("hipRTC: ") + hiprtcGetErrorString(r) + ": " + l;
    hiprtcDestroyProgram(&prog);
    return hipErrorInvalidValue;
  }
  size_t size = 0;
  hiprtcGetCodeSize(prog, &size);
  std::vector<char> code(size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  hipError_t e = hipModuleLoadData(&out->module, code.data());
  if (e != hipSuccess) {
    *log = "hipModuleLoadData";
    return e;
  }
  e = hipModuleGetFunction(&out->fn, out->module, "soax_expr_kernel");
  if (e != hipSuccess) *log = "hipModuleGetFunction";
  return e;
}

}  // namespace

std::string expr_source(const ExprPlan& p) {
  std::vector<double> consts;
  return generate(p, &consts);
}

hipError_t launch_expr(const ExprPlan& p, hipStream_t s, std::string* log) {
  std::vector<double> consts;
  const std::string src = generate(p, &consts);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Compiled c;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_tuple(dev, src);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
      hipDeviceProp_t prop;
      if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return e;
      if ((e = compile(src, prop.gcnArchName, &c, log)) != hipSuccess) return e;
      g_cache[key] = c;
    } else {
      c = it->second;
    }
  }
  if (p.n == 0) return hipSuccess;
  ExprArgs a{};
  for (int j = 0; j < p.nsrc; ++j) a.src[j] = p.src[j];
  a.dst = p.dst;
  a.n = p.n;
  for (size_t j = 0; j < consts.size(); ++j) a.c[j] = consts[j];
  size_t size = sizeof a;
  void* config[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, &a, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size,
                    HIP_LAUNCH_PARAM_END};
  const int64_t per_block = static_cast<int64_t>(kExprBlock) * kExprPerThread;
  const unsigned grid = static_cast<unsigned>((p.n + per_block - 1) / per_block);
  return hipModuleLaunchKernel(c.fn, grid, 1, 1, kExprBlock, 1, 1, 0, s, nullptr, config);
}

}  // namespace soax
