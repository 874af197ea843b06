/*
 * soaxref.h -- CPU oracle for the SoA/AoS particle-update hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct CPU definition.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * Every routine works on host memory, one particle at a time, in fp64
 * (values of narrower fields are widened to double, combined in double and
 * rounded back when stored, which is C's usual arithmetic conversion for a
 * double time step applied to float fields).  Compile with
 * -ffp-contract=off so that every a*b+c is two IEEE roundings.
 *
 * Return value of every int routine: 0 on success, a negative code on bad
 * arguments (-1 argument, -2 schema).  Nothing aborts.
 *
 * Parity unpinned, by design: sin, cos, log and sqrt here are glibc's, and
 * the GPU library evaluates its own, so field values, RK2/Heun/RK4
 * positions and the Box-Muller normals of the fill agree with this oracle
 * within the tests' tolerances, not bit for bit.  Every routine is otherwise
 * pinned by the tests to values the paper or the mathematics fix.
 */
#ifndef SOAXREF_H
#define SOAXREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Field element types (the code values are this oracle's own). */
enum { REF_I8 = 1, REF_U8 = 2, REF_I32 = 3, REF_I64 = 4, REF_F32 = 5, REF_F64 = 6 };

/* Integrators. */
enum {
  REF_EULER = 0,
  REF_EULER_ACC = 1,
  REF_RK2_ABC = 2,
  REF_HEUN_ABC = 3,
  REF_RK4_ABC = 4,
  REF_SYMPLECTIC_EULER = 5
};

/*
 * A particle schema: an ordered list of named properties, each an element
 * type and a dimension 1..3 (the paper's attribute tuple of Section 4.1,
 * Listing "typical usage": id<int,1>, pos<double,3>, ...).
 */
typedef struct {
  int32_t nfields;
  const char* const* names;
  const int32_t* dtypes;
  const int32_t* dims;
  int32_t packed; /* 0: C natural alignment (the AoS struct of Listing 1); 1: no padding */
} ref_schema;

int soaxref_threads(int nthreads); /* set OpenMP threads if >0; returns threads in use */

/* AoS byte offset of each field and the record stride (Section 1, Listing 1). */
int soaxref_layout(const ref_schema* s, int64_t* offsets, int64_t* stride);

/* SplitMix64 (Steele, Lea & Flood 2014): finaliser and counter-based draw. */
uint64_t soaxref_mix64(uint64_t z);
uint64_t soaxref_draw(uint64_t seed, uint64_t stream, uint64_t i);

/*
 * Seeded synthetic fill of the SoA arrays.  soa[a] is the array of
 * component c of field f, a = (sum of dims of fields before f) + c.
 * vel_mode 0: vel ~ N(0,1); 1: vel = field u(pos) with amplitudes abc[3].
 */
int soaxref_fill(const ref_schema* s, int64_t n, uint64_t seed, int vel_mode,
                 const double* abc, void* const* soa);

/* The same values for particles first .. first+n-1 only (soa[a][j] holds
 * particle first + j): every value depends on the particle index alone. */
int soaxref_fill_range(const ref_schema* s, int64_t first, int64_t n, uint64_t seed, int vel_mode,
                       const double* abc, void* const* soa);

/* ABC velocity field u(x) for one point. */
void soaxref_field(const double* abc, const double* x, double* u);

/* Time steps on SoA arrays / on an AoS buffer (record stride from soaxref_layout). */
int soaxref_step_soa(const ref_schema* s, int64_t n, void* const* soa, int integrator,
                     double dt, int64_t nsteps, const double* abc, int wrap);
int soaxref_step_aos(const ref_schema* s, int64_t n, void* aos, int integrator,
                     double dt, int64_t nsteps, const double* abc, int wrap);

/* Remove flagged particles by overwriting each with the last particle
 * (Section 2); returns the new count (negative on bad arguments). */
int64_t soaxref_remove_flagged(const ref_schema* s, int64_t n, void* const* soa, uint8_t* flags);

/* Bulk layout transposes; soa_to_aos writes every padding byte as 0. */
int soaxref_aos_to_soa(const ref_schema* s, int64_t n, const void* aos, void* const* soa);
int soaxref_soa_to_aos(const ref_schema* s, int64_t n, void* const* soa, void* aos);

/* AoSoA (tiled) layout: particles grouped in tiles of REF_AOSOA_W; a tile
 * holds, for every SoA array in order, its REF_AOSOA_W elements back to
 * back, so element i of array a is at byte
 *   (i / W) * tile_bytes + array_offsets[a] + (i % W) * esize(a),
 *   array_offsets[a] = W * (sum of the element sizes of the arrays before a),
 *   tile_bytes = W * (sum of all element sizes).
 * soa_to_aosoa writes ceil(n / W) whole tiles, the unused lanes of the last
 * tile as zero bytes. */
enum { REF_AOSOA_W = 64 };
int soaxref_aosoa_layout(const ref_schema* s, int64_t* array_offsets, int64_t* tile_bytes);
int soaxref_soa_to_aosoa(const ref_schema* s, int64_t n, void* const* soa, void* aosoa);
int soaxref_aosoa_to_soa(const ref_schema* s, int64_t n, const void* aosoa, void* const* soa);

/*
 * RK2 (explicit midpoint) advection without wrap, positions only:
 * x[d][i] in, xT[d][i] out.  states, if not NULL, receives every state
 * x_0..x_nsteps as states[(s*3+d)*n + i].
 */
int soaxref_rk2_forward(int64_t n, const double* const* x0, double* const* xT,
                        const double* abc, double dt, int64_t nsteps, double* states);

/* Loss sum_i sum_d (xT - target)^2 and its gradient lamT = 2 (xT - target). */
double soaxref_sqdist_loss(int64_t n, const double* const* xT, const double* const* target,
                           double* const* lamT);

/*
 * Discrete adjoint of soaxref_rk2_forward (every state stored, then one
 * reverse sweep).  Given lamT = dL/dxT, returns dL/dx0 and dL/d(A,B,C).
 */
int soaxref_adjoint(int64_t n, const double* const* x0, const double* const* lamT,
                    const double* abc, double dt, int64_t nsteps,
                    double* const* grad_x0, double* grad_abc);

/* The same gradients by forward-mode (tangent) propagation of the 3x3 state
 * and parameter Jacobians: an independent algorithm used to pin the adjoint. */
int soaxref_tangent(int64_t n, const double* const* x0, const double* const* lamT,
                    const double* abc, double dt, int64_t nsteps,
                    double* const* grad_x0, double* grad_abc);

#ifdef __cplusplus
}
#endif
#endif
