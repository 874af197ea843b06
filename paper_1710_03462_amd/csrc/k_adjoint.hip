// k_adjoint.hip -- gfx950 kernels for differentiating RK2 advection in the
// ABC field: forward with checkpoints, the discrete adjoint with
// recomputation, and a squared-distance loss.
//
// One thread owns one particle for the whole time loop (the state stays in
// registers).  The adjoint walks the checkpoint segments backwards; for each
// segment it recomputes the states from the checkpoint into a register array
// indexed by compile-time constants (fully unrolled loops, so the array never
// touches scratch memory) and sweeps them backwards.  Segments longer than
// the register array are split into sub-segments, each recomputed from the
// checkpoint.  When k and nsteps are multiples of the renewal interval
// below, the forward and the adjoint run their steps in blocks of straight-
// line code without a branch per step.  Parameter gradients are summed per
// particle in reverse step order, then over particles by a fixed-shape tree
// (per workgroup, then one final workgroup), so results are deterministic and
// do not depend on k.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "launch.h"

namespace soax {

namespace {

constexpr int kRedBlock = kAdjointBlock;  // workgroup size of every reducing kernel



// Rows of one checkpoint on the tape: the position and the sines and cosines
// the forward evaluated at it.
constexpr int kTapeRows = 9;

// Sines and cosines of the state of step s (its global index) in the loops
// over many steps of one particle.  With every step proven small (SMALL)
// they come from the previous state's by angle addition over the step's
// displacement (the difference of the two rounded positions), renewed by a
// full reduction at every step index that is a multiple of kAnchor, so each
// value depends on the step index alone (not on the checkpoint interval) and
// carries at most kAnchor - 1 angle additions (about one ulp of 1 each).
// Larger steps reduce every state in full.  kAnchor equals the register
// block of the usual checkpoint interval (20), so that a block that starts
// at a multiple of it has no renewal inside its recomputation and exactly
// one, at its first reversed state, in the reverse sweep: such blocks run as
// straight-line code (rk2_ckpt_blocks_kernel, adjoint_blocks_kernel).
constexpr int64_t kAnchor = 20;

// The angle-shift tier of these kernels: SMALL (small_steps holds) or any shift.
template <bool SMALL>
constexpr int kTierOf = SMALL ? kTierSmall : kTierAny;

// One explicit-midpoint step from (x, y, z) with sines and cosines t, no
// wrap; on return (x, y, z) is the next state and t its sines and cosines as
// above (renew: the next state's index is a multiple of kAnchor).  (dt/2) k1
// and dt k2 are the fields of the amplitudes scaled by dt/2 and dt, which a
// loop computes once.
template <bool SMALL>
__device__ __forceinline__ void rk2_advance(const Abc& p, double dt, bool renew, double& x,
                                            double& y, double& z, Trig3& t) {
  double m0, m1, m2;
  field_of(scaled(p, 0.5 * dt), t, m0, m1, m2);
  const Trig3 tm = trig3_shift<kTierOf<SMALL>>(t, x, y, z, m0, m1, m2);
  field_of(scaled(p, dt), tm, m0, m1, m2);
  const double x1 = x + m0, y1 = y + m1, z1 = z + m2;
  if (!SMALL || renew)
    t = trig3(x1, y1, z1);
  else
    t = trig3_shift<kTierOf<SMALL>>(t, x, y, z, x1 - x, y1 - y, z1 - z);
  x = x1;
  y = y1;
  z = z1;
}

// rk2_advance<true> for a step whose next state is not a renewal point: the
// same arithmetic without the branch.
__device__ __forceinline__ void rk2_advance_carry(const Abc& p, double dt, double& x, double& y,
                                                  double& z, Trig3& t) {
  double m0, m1, m2;
  field_of(scaled(p, 0.5 * dt), t, m0, m1, m2);
  const Trig3 tm = trig3_shift<kTierSmall>(t, x, y, z, m0, m1, m2);
  field_of(scaled(p, dt), tm, m0, m1, m2);
  const double x1 = x + m0, y1 = y + m1, z1 = z + m2;
  t = trig3_shift<kTierSmall>(t, x, y, z, x1 - x, y1 - y, z1 - z);
  x = x1;
  y = y1;
  z = z1;
}

template <bool SMALL>
__global__ __launch_bounds__(256) void rk2_ckpt_kernel(CkptArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Abc p = to_abc(a.abc);
  const int64_t e = i * a.stride;
  double x = a.x0[0][e], y = a.x0[1][e], z = a.x0[2][e];
  Trig3 t = trig3(x, y, z);
  double* tp = a.tape + i;
  const int64_t n = a.n;
  int64_t until_ckpt = 0;
  int r = 1;  // (s + 1) mod kAnchor, kept by counting
  for (int64_t s = 0; s < a.nsteps; ++s) {
    if (until_ckpt == 0) {  // the tape is written once and read back much later
      st1<true>(tp, x);
      st1<true>(tp + n, y);
      st1<true>(tp + 2 * n, z);
      st1<true>(tp + 3 * n, t.sx);
      st1<true>(tp + 4 * n, t.cx);
      st1<true>(tp + 5 * n, t.sy);
      st1<true>(tp + 6 * n, t.cy);
      st1<true>(tp + 7 * n, t.sz);
      st1<true>(tp + 8 * n, t.cz);
      tp += kTapeRows * n;
      until_ckpt = a.k;
    }
    --until_ckpt;
    rk2_advance<SMALL>(p, a.dt, r == 0, x, y, z, t);
    r = r + 1 == kAnchor ? 0 : r + 1;
  }
  st1<true>(a.xT[0] + e, x);
  st1<true>(a.xT[1] + e, y);
  st1<true>(a.xT[2] + e, z);
}

// rk2_ckpt_kernel<true> when k and nsteps are multiples of kAnchor: the
// steps run in blocks of kAnchor that start at renewal points, each kAnchor
// - 1 carried steps and one renewed step as straight-line code (the same
// values; without a branch per step the compiler overlaps consecutive
// steps).  Every checkpoint falls on a block's start.
__global__ __launch_bounds__(256) void rk2_ckpt_blocks_kernel(CkptArgs a) {
  constexpr int KB = static_cast<int>(kAnchor);
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const Abc p = to_abc(a.abc);
  const int64_t e = i * a.stride;
  double x = a.x0[0][e], y = a.x0[1][e], z = a.x0[2][e];
  Trig3 t = trig3(x, y, z);
  double* tp = a.tape + i;
  const int64_t n = a.n;
  for (int64_t s0 = 0; s0 < a.nsteps; s0 += KB) {
    if (s0 % a.k == 0) {
      st1<true>(tp, x);
      st1<true>(tp + n, y);
      st1<true>(tp + 2 * n, z);
      st1<true>(tp + 3 * n, t.sx);
      st1<true>(tp + 4 * n, t.cx);
      st1<true>(tp + 5 * n, t.sy);
      st1<true>(tp + 6 * n, t.cy);
      st1<true>(tp + 7 * n, t.sz);
      st1<true>(tp + 8 * n, t.cz);
      tp += kTapeRows * n;
    }
#pragma unroll
    for (int j = 0; j < KB - 1; ++j) rk2_advance_carry(p, a.dt, x, y, z, t);
    rk2_advance<true>(p, a.dt, true, x, y, z, t);
  }
  st1<true>(a.xT[0] + e, x);
  st1<true>(a.xT[1] + e, y);
  st1<true>(a.xT[2] + e, z);
}

// Reverse one midpoint step taken from state (x, y, z), whose sines and
// cosines are t.  With xm = x + (dt/2) u(x) and x+ = x + dt u(xm):
//   mu  = dt J(xm)^T lam+
//   g  += dt G(xm)^T lam+ + (dt/2) G(x)^T mu
//   lam = lam+ + mu + (dt/2) J(x)^T mu
// where J = du/dx and G = du/d(A,B,C).
template <bool SMALL>
__device__ __forceinline__ void rk2_reverse(const Abc& p, double dt, const Trig3& t, double x,
                                            double y, double z, double& l0, double& l1,
                                            double& l2, double& g0, double& g1, double& g2) {
  const double h = 0.5 * dt;
  double h0, h1, h2;  // (dt/2) u(x), as in the forward step
  field_of(scaled(p, h), t, h0, h1, h2);
  const Trig3 m = trig3_shift<kTierOf<SMALL>>(t, x, y, z, h0, h1, h2);  // at xm
  // mu = dt J(xm)^T lam, each component an amplitude times one fused
  // difference; dt is folded into the amplitudes
  const double dA = dt * p.A, dB = dt * p.B, dC = dt * p.C;
  const double m0 = dB * fma(m.cx, l1, -(m.sx * l2));
  const double m1 = dC * fma(m.cy, l2, -(m.sy * l0));
  const double m2 = dA * fma(m.cz, l0, -(m.sz * l1));
  // g += dt G(xm)^T lam + (dt/2) G(x)^T mu
  const double qa = fma(m.sz, l0, m.cz * l1), qb = fma(m.sx, l1, m.cx * l2),
               qc = fma(m.cy, l0, m.sy * l2);
  const double ra = fma(t.sz, m0, t.cz * m1), rb = fma(t.sx, m1, t.cx * m2),
               rc = fma(t.cy, m0, t.sy * m2);
  g0 = g0 + fma(dt, qa, h * ra);
  g1 = g1 + fma(dt, qb, h * rb);
  g2 = g2 + fma(dt, qc, h * rc);
  // lam = lam+ + mu + (dt/2) J(x)^T mu, with dt/2 folded into the amplitudes
  const double hA = h * p.A, hB = h * p.B, hC = h * p.C;
  l0 = (l0 + m0) + hB * fma(t.cx, m1, -(t.sx * m2));
  l1 = (l1 + m1) + hC * fma(t.cy, m2, -(t.sy * m0));
  l2 = (l2 + m2) + hA * fma(t.cz, m0, -(t.sz * m1));
}

// With every step proven small (SMALL), the reverse sweep takes the sines
// and cosines of each state from those of the state one step later (reversed
// just before it) by angle addition over the difference of the two
// positions, renewed by a full reduction at the last step and at every step
// whose index is kAnchor - 1 modulo kAnchor; like the forward's, these values
// depend on the step index alone.  Larger steps reduce every state in full.

// Sum v over the workgroup (kRedBlock threads) in a fixed tree order.
__device__ __forceinline__ void block_sum3(double v0, double v1, double v2, double* out3) {
  __shared__ double red[3][kRedBlock];
  const int t = threadIdx.x;
  red[0][t] = v0;
  red[1][t] = v1;
  red[2][t] = v2;
  __syncthreads();
  for (int s = kRedBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
      red[2][t] += red[2][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out3[0] = red[0][0];
    out3[1] = red[1][0];
    out3[2] = red[2][0];
  }
}

// KM: states held in registers per (sub-)segment.
template <int KM, bool SMALL>
__global__ __launch_bounds__(kRedBlock) void adjoint_kernel(AdjointArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const Abc p = to_abc(a.abc);
  const double dt = a.dt;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (i < a.n) {
    const int64_t n = a.n;
    const int64_t e = i * a.stride;
    double l0 = a.lam[0][e], l1 = a.lam[1][e], l2 = a.lam[2][e];
    const int64_t nseg = (a.nsteps + a.k - 1) / a.k;
    Trig3 tn{};  // sines and cosines of the state reversed last, at (xn, yn, zn)
    double xn = 0.0, yn = 0.0, zn = 0.0;
    for (int64_t c = nseg - 1; c >= 0; --c) {
      const int64_t len = min(a.k, a.nsteps - c * a.k);
      const double* cp = a.tape + (c * kTapeRows) * n + i;
      const int64_t nsub = (len + KM - 1) / KM;
      for (int64_t q = nsub - 1; q >= 0; --q) {
        double x = cp[0], y = cp[n], z = cp[2 * n];
        Trig3 t{cp[3 * n], cp[4 * n], cp[5 * n], cp[6 * n], cp[7 * n], cp[8 * n]};
        // r: (index of the state after the next step) mod kAnchor, by counting
        int r = static_cast<int>((c * a.k + 1) % kAnchor);
        for (int64_t s = c * a.k; s < c * a.k + q * KM; ++s) {
          rk2_advance<SMALL>(p, dt, r == 0, x, y, z, t);
          r = r + 1 == kAnchor ? 0 : r + 1;
        }
        const int m = static_cast<int>(min(static_cast<int64_t>(KM), len - q * KM));
        double sx[KM], sy[KM], sz[KM];
#pragma unroll
        for (int j = 0; j < KM; ++j) {
          if (j < m) {
            sx[j] = x;
            sy[j] = y;
            sz[j] = z;
            if (j + 1 < m) rk2_advance<SMALL>(p, dt, r == 0, x, y, z, t);
            r = r + 1 == kAnchor ? 0 : r + 1;
          }
        }
        const int64_t t0 = c * a.k + q * KM;  // global index of state 0
        const int r0 = static_cast<int>(t0 % kAnchor);
#pragma unroll
        for (int j = KM - 1; j >= 0; --j) {
          if (j < m) {
            const int64_t ts = t0 + j;
            int rj = r0 + j;  // ts mod kAnchor (r0 + j < 3 kAnchor)
            if (rj >= kAnchor) rj -= kAnchor;
            if (rj >= kAnchor) rj -= kAnchor;
            Trig3 tj;
            if (!SMALL || ts == a.nsteps - 1 || rj == kAnchor - 1)
              tj = trig3(sx[j], sy[j], sz[j]);
            else
              tj = trig3_shift<kTierOf<SMALL>>(tn, xn, yn, zn, sx[j] - xn, sy[j] - yn, sz[j] - zn);
            rk2_reverse<SMALL>(p, dt, tj, sx[j], sy[j], sz[j], l0, l1, l2, g0, g1, g2);
            tn = tj;
            xn = sx[j];
            yn = sy[j];
            zn = sz[j];
          }
        }
      }
    }
    a.gx[0][e] = l0;
    a.gx[1][e] = l1;
    a.gx[2][e] = l2;
  }
  block_sum3(g0, g1, g2, a.partial + 3 * static_cast<int64_t>(blockIdx.x));
}

// The adjoint when every step is small and both k and nsteps are multiples
// of kAnchor: every segment's length is then a multiple of kAnchor too, and
// every block of kAnchor states starts at a renewal point (its first
// state's index is a multiple of kAnchor).  Its states t0 + 1 ..
// t0 + kAnchor - 1 are not renewal points, so the recomputation only carries;
// the reverse sweep renews at the block's last state (index kAnchor - 1
// modulo kAnchor) and carries down from there.  These are adjoint_kernel's
// values bit for bit, as straight-line code without a branch per step, which
// lets the compiler overlap consecutive steps (adjoint_kernel's per-step
// branches split the code into blocks it does not schedule across).
__global__ __launch_bounds__(kRedBlock) void adjoint_blocks_kernel(AdjointArgs a) {
  constexpr int KB = static_cast<int>(kAnchor);
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const Abc p = to_abc(a.abc);
  const double dt = a.dt;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (i < a.n) {
    const int64_t n = a.n;
    const int64_t e = i * a.stride;
    double l0 = a.lam[0][e], l1 = a.lam[1][e], l2 = a.lam[2][e];
    const int64_t nseg = (a.nsteps + a.k - 1) / a.k;
    for (int64_t c = nseg - 1; c >= 0; --c) {
      // k and nsteps are multiples of KB, so every segment's length is too
      const int64_t len = min(a.k, a.nsteps - c * a.k);
      const double* cp = a.tape + (c * kTapeRows) * n + i;
      for (int64_t q = len / KB - 1; q >= 0; --q) {
        double x = cp[0], y = cp[n], z = cp[2 * n];
        Trig3 t{cp[3 * n], cp[4 * n], cp[5 * n], cp[6 * n], cp[7 * n], cp[8 * n]};
        int r = 1;  // c k is a multiple of kAnchor; (s + 1) mod kAnchor by counting
        for (int64_t s = c * a.k; s < c * a.k + q * KB; ++s) {
          rk2_advance<true>(p, dt, r == 0, x, y, z, t);
          r = r + 1 == KB ? 0 : r + 1;
        }
        double bx[KB], by[KB], bz[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
          bx[j] = x;
          by[j] = y;
          bz[j] = z;
          if (j + 1 < KB) rk2_advance_carry(p, dt, x, y, z, t);
        }
        Trig3 tj = trig3(bx[KB - 1], by[KB - 1], bz[KB - 1]);
        rk2_reverse<true>(p, dt, tj, bx[KB - 1], by[KB - 1], bz[KB - 1], l0, l1, l2, g0, g1, g2);
#pragma unroll
        for (int j = KB - 2; j >= 0; --j) {
          tj = trig3_shift<kTierSmall>(tj, bx[j + 1], by[j + 1], bz[j + 1], bx[j] - bx[j + 1],
                                       by[j] - by[j + 1], bz[j] - bz[j + 1]);
          rk2_reverse<true>(p, dt, tj, bx[j], by[j], bz[j], l0, l1, l2, g0, g1, g2);
        }
      }
    }
    a.gx[0][e] = l0;
    a.gx[1][e] = l1;
    a.gx[2][e] = l2;
  }
  block_sum3(g0, g1, g2, a.partial + 3 * static_cast<int64_t>(blockIdx.x));
}

// One workgroup: out[d] = sum_b partial[3b + d], each thread summing a fixed
// strided slice in order, then the fixed tree.
__global__ __launch_bounds__(kRedBlock) void final_sum3_kernel(const double* __restrict__ partial,
                                                               int64_t nparts,
                                                               double* __restrict__ out) {
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += kRedBlock) {
    v0 += partial[3 * b];
    v1 += partial[3 * b + 1];
    v2 += partial[3 * b + 2];
  }
  block_sum3(v0, v1, v2, out);
}

// Like final_sum3_kernel but the sum of the three components goes to out[0].
__global__ __launch_bounds__(kRedBlock) void final_sum1_kernel(const double* __restrict__ partial,
                                                               int64_t nparts,
                                                               double* __restrict__ out) {
  __shared__ double tot[3];
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += kRedBlock) {
    v0 += partial[3 * b];
    v1 += partial[3 * b + 1];
    v2 += partial[3 * b + 2];
  }
  block_sum3(v0, v1, v2, tot);
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (tot[0] + tot[1]) + tot[2];
}

__global__ __launch_bounds__(kRedBlock) void sqdist_kernel(LossArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  if (i < a.n) {
    const int64_t e = i * a.stride;
    e0 = a.xT[0][e] - a.target[0][i];
    e1 = a.xT[1][e] - a.target[1][i];
    e2 = a.xT[2][e] - a.target[2][i];
    if (a.lam[0]) {
      a.lam[0][e] = 2.0 * e0;
      a.lam[1][e] = 2.0 * e1;
      a.lam[2][e] = 2.0 * e2;
    }
  }
  block_sum3(e0 * e0, e1 * e1, e2 * e2, a.partial + 3 * static_cast<int64_t>(blockIdx.x));
}

}  // namespace

hipError_t launch_rk2_forward_ckpt(const CkptArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t grid = (a.n + 255) / 256;
  const bool small = small_steps(a.dt, a.abc.A, a.abc.B, a.abc.C);
  if (small && a.k % kAnchor == 0 && a.nsteps % kAnchor == 0)
    hipLaunchKernelGGL(rk2_ckpt_blocks_kernel, dim3(grid), dim3(256), 0, s, a);
  else if (small)
    hipLaunchKernelGGL(rk2_ckpt_kernel<true>, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rk2_ckpt_kernel<false>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

int64_t adjoint_partials(int64_t n) { return (n + kRedBlock - 1) / kRedBlock; }

hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t s) {
  const int64_t grid = adjoint_partials(a.n);
  if (grid > 0) {
    const bool small = small_steps(a.dt, a.abc.A, a.abc.B, a.abc.C);
    if (small && a.k % kAnchor == 0 && a.nsteps % kAnchor == 0) {
      hipLaunchKernelGGL(adjoint_blocks_kernel, dim3(grid), dim3(kRedBlock), 0, s, a);
    } else if (small) {
      if (a.k <= 8)
        hipLaunchKernelGGL((adjoint_kernel<8, true>), dim3(grid), dim3(kRedBlock), 0, s, a);
      else if (a.k <= 20)
        hipLaunchKernelGGL((adjoint_kernel<20, true>), dim3(grid), dim3(kRedBlock), 0, s, a);
      else
        hipLaunchKernelGGL((adjoint_kernel<32, true>), dim3(grid), dim3(kRedBlock), 0, s, a);
    } else {
      if (a.k <= 8)
        hipLaunchKernelGGL((adjoint_kernel<8, false>), dim3(grid), dim3(kRedBlock), 0, s, a);
      else if (a.k <= 20)
        hipLaunchKernelGGL((adjoint_kernel<20, false>), dim3(grid), dim3(kRedBlock), 0, s, a);
      else
        hipLaunchKernelGGL((adjoint_kernel<32, false>), dim3(grid), dim3(kRedBlock), 0, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(final_sum3_kernel, dim3(1), dim3(kRedBlock), 0, s, a.partial, grid,
                     a.grad_abc);
  return hipGetLastError();
}

int64_t loss_partials(int64_t n) { return (n + kRedBlock - 1) / kRedBlock; }

hipError_t launch_sqdist_loss(const LossArgs& a, hipStream_t s) {
  const int64_t grid = loss_partials(a.n);
  if (grid > 0) {
    hipLaunchKernelGGL(sqdist_kernel, dim3(grid), dim3(kRedBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(final_sum1_kernel, dim3(1), dim3(kRedBlock), 0, s, a.partial, grid, a.loss);
  return hipGetLastError();
}

}  // namespace soax
