// launch.h -- interface between the host side of the C ABI (soax_host.cpp)
// and the kernel translation units.  Launchers validate nothing: the host
// side has already checked sizes, types and alignment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace soax {

struct Abc;

constexpr int kMaxFields = 32;
constexpr int kMaxArrays = 3 * kMaxFields;

// Element type codes (same values as soax_dtype).
enum Dtype : int32_t { kI8 = 1, kU8 = 2, kI32 = 3, kI64 = 4, kF32 = 5, kF64 = 6 };
enum Integrator : int32_t {
  kEuler = 0, kEulerAcc = 1, kRk2Abc = 2, kHeunAbc = 3, kRk4Abc = 4, kSymEuler = 5
};
// Integrators that evaluate the ABC field (need f64 positions and amplitudes).
constexpr bool field_integrator(int i) { return i == kRk2Abc || i == kHeunAbc || i == kRk4Abc; }
// Integrators that read an acceleration property.
constexpr bool uses_acc(int i) { return i == kEulerAcc || i == kSymEuler; }

inline int dtype_size(int32_t t) {
  switch (t) {
    case kI8: case kU8: return 1;
    case kI32: case kF32: return 4;
    case kI64: case kF64: return 8;
    default: return 0;
  }
}

struct AbcParams {
  double A, B, C;
};

// Largest displacement per coordinate for which a step's midpoint and end
// point sines come from its start point by angle addition without a check.
constexpr double kShiftLimit = 1.0 / 64;

// True when every displacement of a midpoint step, (dt/2) u and dt u, is at
// most kShiftLimit in each coordinate, since |u_i| <= |A| + |B| + |C|.
inline __host__ __device__ bool small_steps(double dt, double A, double B, double C) {
  const double s = (A < 0 ? -A : A) + (B < 0 ? -B : B) + (C < 0 ? -C : C);
  return (dt < 0 ? -dt : dt) * s <= kShiftLimit;
}

// What the host proves about every displacement of a step of the field
// integrators (the shift of the angle additions): kTierSmall, every shift at
// most kShiftLimit (the short series); kTierMid, every shift at most 1/8 (the
// longer series; checked against kShiftMidLimit, 1/8 less 2^-20 of it, so
// that no rounding of dt u can carry a shift past 1/8); kTierAny, no bound.
// The tier is a function of dt and the amplitudes alone, so every layout, the
// batch and the single-set kernels take the same one for the same step; the
// mid-tier kernels give exactly the results of the kTierAny kernels on every
// step that satisfies their bound.
enum ShiftTier : int32_t { kTierSmall = 0, kTierMid = 1, kTierAny = 2 };
constexpr double kShiftMidLimit = 0.125 * (1.0 - 0x1p-20);

inline __host__ __device__ int shift_tier(double dt, double A, double B, double C) {
  const double s = (A < 0 ? -A : A) + (B < 0 ? -B : B) + (C < 0 ? -C : C);
  const double m = (dt < 0 ? -dt : dt) * s;
  return m <= kShiftLimit ? kTierSmall : (m <= kShiftMidLimit ? kTierMid : kTierAny);
}

// A step whose arrays span at least this many bytes streams through HBM and
// uses nontemporal hints; smaller working sets stay cache-resident between
// steps and use ordinary accesses.
constexpr int64_t kStreamBytes = int64_t(128) << 20;

// Bytes of one particle the SoA step reads or writes: positions and
// velocities, plus the acceleration for the integrators that use it.
inline int64_t soa_step_bytes(int integ, int pos_size, int vel_size) {
  return 3 * (pos_size + vel_size) + (uses_acc(integ) ? 3 * vel_size : 0);
}

// ------------------------------------------------------------------ steps

struct SoaStepArgs {
  void* pos[3];
  void* vel[3];
  const void* acc[3];  // Euler-with-acceleration only; same type as vel
  int64_t n;
  double dt;
  AbcParams abc;
  int32_t wrap;
};

// vec = particles per thread (1, 2, 4; 2 and 4 need 16-byte aligned arrays).
hipError_t launch_soa_step(int integ, int pos_t, int vel_t, int vec, int block,
                           const SoaStepArgs& a, hipStream_t s);

// nsteps (>= 1) steps of integ in one launch, each particle held in registers
// from the first step to the last (one thread per particle).
hipError_t launch_soa_fused(int integ, int pos_t, int vel_t, int block, const SoaStepArgs& a,
                            int64_t nsteps, hipStream_t s);

struct AosStepArgs {
  char* aos;
  int64_t n;
  int32_t stride;
  int32_t off_pos, off_vel, off_acc;
  double dt;
  AbcParams abc;
  int32_t wrap;
};

// LDS-staged tile kernel: needs a 16-byte aligned buffer; `aligned` says
// every pos/vel/acc element is naturally aligned inside a record.
hipError_t launch_aos_step(int integ, int pos_t, int vel_t, bool aligned, int block,
                           const AosStepArgs& a, hipStream_t s);
// One thread per record, direct per-field global accesses.
hipError_t launch_aos_naive(int integ, int pos_t, int vel_t, bool aligned, int block,
                            const AosStepArgs& a, hipStream_t s);
// Largest tile (records) whose LDS staging fits the per-block budget.
int aos_tile_records(int stride, int block);

// -------------------------------------------------------------- transposes

struct XposeArgs {
  char* aos;
  int64_t n;  // particles to move; the kernels take it as an argument, not from the table
  int32_t stride;
  int32_t narrays;
  int32_t aligned;  // every element naturally aligned inside the record
  char* soa[kMaxArrays];
  int32_t off[kMaxArrays];  // byte offset of the element inside the record
  int32_t es[kMaxArrays];   // element size
  int32_t order[kMaxArrays];  // array indices grouped by size: 8-byte, 4-byte, then 1-byte
  int32_t group_end[3];       // end of each size's group in order[]
};

// Fill order and group_end from es[0..narrays) (element sizes 8, 4 or 1).
inline void group_by_size(XposeArgs& t) {
  const int32_t sizes[3] = {8, 4, 1};
  int k = 0;
  for (int g = 0; g < 3; ++g) {
    for (int a = 0; a < t.narrays; ++a)
      if (t.es[a] == sizes[g]) t.order[k++] = a;
    t.group_end[g] = k;
  }
}

// `host` is a host copy of the table the kernels read from `dev` (device
// memory, uploaded when the set's buffers change); host.n is passed by value.
hipError_t launch_xpose(bool to_soa, const XposeArgs& host, const XposeArgs* dev, hipStream_t s);

// AoSoA tiles of kAosoaW particles: a tile holds every SoA array's kAosoaW
// elements back to back.  The conversions use an XposeArgs table with
// aos = the tiled buffer, stride = bytes per tile and off[a] = the offset of
// array a inside a tile; soa -> aosoa writes the unused lanes of the last
// tile as zero bytes.
constexpr int kAosoaW = 64;
hipError_t launch_aosoa_xpose(bool to_soa, const XposeArgs& host, const XposeArgs* dev,
                              hipStream_t s);

struct AosoaStepArgs {
  char* base;          // tiled buffer
  int64_t tile_bytes;
  int32_t off_pos[3];  // offsets of the component arrays inside a tile
  int32_t off_vel[3];
  int32_t off_acc[3];
  int64_t n;
  double dt;
  AbcParams abc;
  int32_t wrap;
};
hipError_t launch_aosoa_step(int integ, int pos_t, int vel_t, int block, const AosoaStepArgs& a,
                             hipStream_t s);

// -------------------------------------------------------------------- fill

enum FillRule : int32_t {
  kFillIndex = 0,     // i
  kFillRaw = 1,       // low bytes of the draw
  kFillTop8 = 2,      // draw >> 56
  kFillBox = 3,       // L * U[0,1)
  kFillNormal = 4,    // Box-Muller N(0,1) from streams s and s+1
  kFillMass = 5,      // 0.5 + 1.5 * U[0,1)
  kFillUnit = 6,      // U[0,1)
};

struct FillArgs {
  void* arr;
  int64_t n;
  uint64_t seed;
  uint64_t stream;
  int32_t dtype;
  int32_t rule;
};

hipError_t launch_fill(const FillArgs& a, hipStream_t s);
// vel = u(pos) (vel_mode 1 of the fill).
hipError_t launch_vel_from_field(int pos_t, int vel_t, const SoaStepArgs& a, hipStream_t s);

// --------------------------------------------------------------- utilities

hipError_t launch_copy16(void* dst, const void* src, int64_t bytes, hipStream_t s);

// Access patterns of the streaming SoA steps without their arithmetic (the
// values of the soax_probe patterns).
enum ProbePattern : int32_t { kProbeRk2 = 0, kProbeEuler = 1, kProbeRead = 2, kProbeWrite = 3 };
struct ProbeArgs {
  double* pos[3];
  float* vel[3];
  int64_t n;
  double c;
};
hipError_t launch_stream_probe(int pattern, const ProbeArgs& a, hipStream_t s);

// --------------------------------------------------------------- adjoint

// Position-like arrays (x0, xT, lam, gx) are read at element i * stride:
// stride 1 for SoA arrays, the record stride in doubles for positions kept
// inside AoS records.  The tape is always [segment][3][n].
struct CkptArgs {
  const double* x0[3];
  double* xT[3];
  double* tape;
  int64_t stride;
  int64_t n;
  int64_t nsteps;
  int64_t k;
  double dt;
  AbcParams abc;
};
hipError_t launch_rk2_forward_ckpt(const CkptArgs& a, hipStream_t s);

// Workgroup size of the adjoint and loss kernels: one partial sum of the
// parameter gradient per kAdjointBlock particles.
constexpr int kAdjointBlock = 256;

struct AdjointArgs {
  const double* tape;
  const double* lam[3];
  double* gx[3];
  int64_t stride;
  double* partial;  // [nblocks][3] per-block parameter-gradient sums
  double* grad_abc;
  int64_t n;
  int64_t nsteps;
  int64_t k;
  double dt;
  AbcParams abc;
};
// number of per-block partial sums launch_adjoint needs (3 doubles each)
int64_t adjoint_partials(int64_t n);
hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t s);

struct LossArgs {
  const double* xT[3];
  const double* target[3];  // SoA (stride 1)
  double* lam[3];
  int64_t stride;           // of xT and lam
  double* partial;
  double* loss;
  int64_t n;
};
int64_t loss_partials(int64_t n);
hipError_t launch_sqdist_loss(const LossArgs& a, hipStream_t s);

// ------------------------------------------------------------- containers

// Removal with overwrite-by-last in three passes over a flag array (one
// byte per particle, nonzero = remove) split into tiles of
// container_tile_size() particles.
int64_t container_tile_size();
int64_t container_tiles(int64_t n);
// counts[b] = flagged particles in tile b.
hipError_t launch_count_flags(const uint8_t* flags, int64_t n, int32_t* counts, hipStream_t s);
// With holes_before[b] = flagged particles in tiles before b and
// movers_after[b] = unflagged particles in tiles after b: hole_at[k] = k-th
// flagged slot below n_new (ascending), mover_at[k] = k-th unflagged particle
// at or above n_new counted from the end, and *nmoves = flagged slots below
// n_new.  Both lists need min(n - n_new, n_new) entries.
hipError_t launch_rank_flags(const uint8_t* flags, int64_t n, int64_t n_new,
                             const int64_t* holes_before, const int64_t* movers_after,
                             int64_t* hole_at, int64_t* mover_at, int64_t* nmoves, hipStream_t s);
// Every array of a set moved by one launch: for k < *nmoves and every listed
// array, element hole_at[k] <- element mover_at[k], `stride` bytes moved
// `word` bytes at a time (word in {1, 4, 8, 16} divides stride and the
// array's alignment).
struct MoveArgs {
  int32_t narrays;
  char* base[kMaxArrays + 1];
  int32_t stride[kMaxArrays + 1];
  int32_t word[kMaxArrays + 1];
};
hipError_t launch_move_all(const MoveArgs& m, const int64_t* hole_at, const int64_t* mover_at,
                           const int64_t* nmoves, int64_t max_moves, hipStream_t s);
// p[0, bytes) = 0.
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);

// ------------------------------------------------------------ expressions

// Fused element-wise expression: dst[i] = program(src...[i]), i < n.  Op codes
// have the values of the soax_expr_op codes.
enum ExprOpCode : int32_t {
  kOpArray = 0, kOpConst = 1, kOpAdd = 2, kOpSub = 3, kOpMul = 4, kOpDiv = 5,
  kOpNeg = 6, kOpAbs = 7, kOpSqrt = 8, kOpMin = 9, kOpMax = 10
};
constexpr int kExprMaxOps = 64;
constexpr int kExprMaxSrc = 8;
constexpr int kExprMaxConst = 32;

struct ExprOp {
  int32_t op, arg;
  double value;
};

// A validated program: every kOpArray arg < nsrc, at most kExprMaxConst
// constants, the stack never underflows and ends with one value.
struct ExprPlan {
  int nops;
  ExprOp ops[kExprMaxOps];
  int nsrc;
  const void* src[kExprMaxSrc];
  int32_t src_t[kExprMaxSrc];
  void* dst;
  int32_t dst_t;
  int64_t n;
  bool stream;  // nontemporal loads and stores
};

// Compiles the program's kernel on first use (hipRTC, cached per program
// shape and device) and launches it; a compiler message goes to *log.
hipError_t launch_expr(const ExprPlan& p, hipStream_t s, std::string* log);
// The generated source (for inspection and tests).
std::string expr_source(const ExprPlan& p);

// -------------------------------------------------------------- batching

struct BatchSet {
  double* pos[3];
  void* vel[3];
  int64_t n;
  int64_t tile_begin;  // first tile of this set in the batch's tile list
  double dt;
  double A, B, C;
  int32_t tier;   // shift_tier of this set's dt and amplitudes
  int32_t reserved;
};

struct BatchLaunch {
  const BatchSet* sets;   // device table
  const int32_t* tile_set;  // device: set index of every tile
  int64_t ntiles;
  int32_t nsets;
  int32_t tile;       // particles per tile = block * per_thread
  int32_t block;
  int32_t per_thread;
  int32_t grid;
  int32_t vel_t;
  int32_t max_tier;  // the largest shift tier of any set (the kernel handles tiers up to it)
};
hipError_t launch_batch_rk2(const BatchLaunch& b, hipStream_t s);

}  // namespace soax
