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

// Straight-line source of one program; `consts` receives the constant values
// in the order the source refers to them.
std::string generate(const ExprPlan& p, std::vector<double>* consts) {
  std::string s;
  char buf[256];
  s += "struct Args { const void* src[" + std::to_string(kExprMaxSrc) +
       "]; void* dst; long long n; double c[" + std::to_string(kExprMaxConst) + "]; };\n";
  s += "extern \"C\" __global__ void __launch_bounds__(256) soax_expr_kernel(Args a) {\n";
  s += "  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;\n";
  s += "  if (i >= a.n) return;\n";
  std::vector<bool> used(kExprMaxSrc, false);
  for (int k = 0; k < p.nops; ++k)
    if (p.ops[k].op == kOpArray) used[p.ops[k].arg] = true;
  for (int j = 0; j < p.nsrc; ++j) {
    if (!used[j]) continue;
    const char* t = ctype(p.src_t[j]);
    if (p.stream)
      snprintf(buf, sizeof buf, "  const double s%d = (double)__builtin_nontemporal_load((const %s*)a.src[%d] + i);\n",
               j, t, j);
    else
      snprintf(buf, sizeof buf, "  const double s%d = (double)((const %s*)a.src[%d])[i];\n", j, t, j);
    s += buf;
  }
  std::vector<std::string> stack;
  for (int k = 0; k < p.nops; ++k) {
    const ExprOp& o = p.ops[k];
    std::string v = "t" + std::to_string(k);
    if (o.op == kOpArray) {
      stack.push_back("s" + std::to_string(o.arg));
      continue;
    }
    if (o.op == kOpConst) {
      stack.push_back("a.c[" + std::to_string(consts->size()) + "]");
      consts->push_back(o.value);
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
  const char* dt = ctype(p.dst_t);
  if (p.stream)
    snprintf(buf, sizeof buf, "  __builtin_nontemporal_store((%s)(%s), (%s*)a.dst + i);\n}\n", dt,
             stack.back().c_str(), dt);
  else
    snprintf(buf, sizeof buf, "  ((%s*)a.dst)[i] = (%s)(%s);\n}\n", dt, dt, stack.back().c_str());
  s += buf;
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
  const unsigned grid = static_cast<unsigned>((p.n + 255) / 256);
  return hipModuleLaunchKernel(c.fn, grid, 1, 1, 256, 1, 1, 0, s, nullptr, config);
}

}  // namespace soax
