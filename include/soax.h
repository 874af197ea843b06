/*
 * soax.h -- C ABI of the MI355X (gfx950) particle-update library.
 *
 * A set of n particles has a user schema: an ordered list of named
 * properties, each with an element type and a dimension (the attribute tuple
 * of Section 4.1, usage listing: id<int,1>, pos<double,3>, vel<...,3>, ...).
 * The set keeps two copies of its records side by side in device memory:
 *
 *   SoA  one contiguous array per (property, component) -- the "structure of
 *        arrays" of Section 1 (Listings 2-3), with each vector component in
 *        its own array as in the benchmark of Section 2;
 *   AoS  one contiguous array of C records laid out like the struct of
 *        Section 1 (Listing 1) -- natural C alignment (each member at a
 *        multiple of its size, record size a multiple of the largest member),
 *        or packed with no padding.
 *
 * All pointers passed to or returned from the library are device pointers
 * unless a parameter says "host".  Every call that touches the device
 * enqueues its work on `stream` (a hipStream_t; NULL is the null stream)
 * and returns without synchronising, except where stated.  The library never
 * aborts or throws: every function returns a soax_status, and
 * soax_last_error() gives a thread-local message for the last failure.
 * Arguments are validated on the host before any device call; an invalid
 * call changes nothing.
 */
#ifndef SOAX_H
#define SOAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t soax_status;
#define SOAX_OK 0
#define SOAX_E_ARG (-1)    /* null pointer, negative size, non-finite dt/amplitude, bad enum */
#define SOAX_E_SCHEMA (-2) /* bad dtype/dim/name, duplicate name, missing pos/vel/acc */
#define SOAX_E_RANGE (-3)  /* n too large for the schema (int32 id, 2^31-1 records) */
#define SOAX_E_LAYOUT (-4) /* the requested layout's buffer is absent or misaligned */
#define SOAX_E_OOM (-5)    /* device allocation failed */
#define SOAX_E_HIP (-6)    /* a HIP runtime call failed (message has hipGetErrorString) */
#define SOAX_E_STATE (-7)  /* operation not valid for this object (e.g. tuning a batch mid-capture) */

/* Element types. */
typedef enum { SOAX_I8 = 1, SOAX_U8 = 2, SOAX_I32 = 3, SOAX_I64 = 4, SOAX_F32 = 5, SOAX_F64 = 6 } soax_dtype;

/* One property: `name` (<= 31 chars, unique), element type, dimension 1..3,
 * and a free one-character descriptive tag (the character argument of the
 * attribute macro of Section 4.2, which the library stores and ignores). */
typedef struct {
  const char* name;
  int32_t dtype;
  int32_t dim;
  char tag;
} soax_field;

/* Ordered property list (1..32 fields); packed = 0 gives C natural alignment. */
typedef struct {
  const soax_field* fields;
  int32_t nfields;
  int32_t packed;
} soax_schema;

/* SOAX_AOSOA: the optional tiled copy (see soax_bind_aosoa). */
typedef enum { SOAX_SOA = 0, SOAX_AOS = 1, SOAX_AOS_NAIVE = 2, SOAX_AOSOA = 3 } soax_layout;

/*
 * Integrators.  Properties are found by name: "pos" (dim 3, f32 or f64),
 * "vel" (dim 3, f32 or f64), "acc" (dim 3, f32 or f64).
 *   SOAX_EULER      pos += dt * vel                                  (Section 2, eq. (1))
 *   SOAX_EULER_ACC  pos += dt * vel with the old vel, then vel += dt * acc
 *   SOAX_RK2_ABC    explicit midpoint in the ABC field
 *                   u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x):
 *                   xm = x + (dt/2) u(x); x = x + dt u(xm); vel = u(x)   (pos must be f64)
 *   SOAX_HEUN_ABC   Heun's rule (explicit trapezoid) in the same field:
 *                   k1 = u(x), k2 = u(x + dt k1); x += (dt/2)(k1 + k2); vel = u(x)
 *   SOAX_RK4_ABC    classical fourth-order Runge-Kutta in the same field;
 *                   vel = u(x) at the new position
 *   SOAX_SYMPLECTIC_EULER  vel += dt * acc first (rounded to vel's type),
 *                   then pos += dt * vel with the new vel
 * Each step is one full pass over the particles.  A double dt applied to a
 * float property is evaluated in double and rounded on store (C's usual
 * arithmetic conversions); no operation is fused into an FMA except in the
 * field integrators' evaluation of the field (the sines and cosines and the
 * sums of amplitude products), so Euler steps are exact to the last bit.
 */
typedef enum {
  SOAX_EULER = 0,
  SOAX_EULER_ACC = 1,
  SOAX_RK2_ABC = 2,
  SOAX_HEUN_ABC = 3,
  SOAX_RK4_ABC = 4,
  SOAX_SYMPLECTIC_EULER = 5
} soax_integrator;

/* Field amplitudes and the periodic wrap of positions into [0, 2*pi)^3
 * (wrap = 1 requires f64 positions: x >= L -> x - L, x < 0 -> x + L, and a
 * sum that rounds to L is stored as 0). */
typedef struct {
  double A, B, C;
  int32_t wrap;
} soax_params;

typedef struct soax_set soax_set;
typedef struct soax_batch soax_batch;

/* ---------------------------------------------------------------- schema */

/*
 * Host only (no device call).  Writes the AoS byte offset of every field
 * (field_offsets[nfields], may be NULL), the AoS record stride and the SoA
 * bytes per particle (sum of element size * dim; either may be NULL).
 */
soax_status soax_schema_layout(const soax_schema* schema, int64_t* field_offsets,
                               int64_t* aos_stride, int64_t* soa_bytes);

/* ------------------------------------------------------------ particle sets */

/*
 * Create a set of n particles on the current HIP device (the container of
 * Section 4.1 constructed for a given particle count, one array per property
 * and component), allocating both layouts (library-owned; freed by
 * soax_destroy).  Each SoA array starts on
 * a 256-byte boundary.  Contents are undefined until filled or written.
 * Errors: ARG (null, n < 0), SCHEMA, RANGE (n > 2^31-1, or an int32/i8/u8
 * "id" too narrow for n), OOM.
 */
soax_status soax_create(const soax_schema* schema, int64_t n, soax_set** out);

/*
 * Wrap caller-owned device memory (e.g. torch tensors) as a set.  soa_ptrs
 * holds one pointer per (field, component) in schema order (the array of
 * component c of field f is at index sum(dims of fields before f) + c); the
 * whole soa_ptrs argument may be NULL (no SoA copy), and aos_ptr may be NULL
 * (no AoS copy).  The library never frees bound memory; the caller keeps it
 * alive until soax_destroy.  Vector (16-byte) kernels are used when every
 * pointer is 16-byte aligned, scalar ones otherwise.
 */
soax_status soax_bind(const soax_schema* schema, int64_t n, void* const* soa_ptrs, void* aos_ptr,
                      soax_set** out);

/* soax_bind for buffers with room for `capacity` >= n particles (each SoA
 * array capacity elements, the AoS buffer capacity records), so that the set
 * can grow up to capacity in place (soax_resize, soax_push_back).  soax_bind
 * is this call with capacity = n. */
soax_status soax_bind_capacity(const soax_schema* schema, int64_t n, int64_t capacity,
                               void* const* soa_ptrs, void* aos_ptr, soax_set** out);

/* Free a set (and the memory it owns).  NULL is ignored.  Does not sync. */
void soax_destroy(soax_set* set);

/* Same as soax_schema_layout for the set's schema. */
soax_status soax_layout_info(const soax_set* set, int64_t* field_offsets, int64_t* aos_stride,
                             int64_t* soa_bytes);

/* Device pointers of the set's buffers: array `index` of the SoA copy (see
 * soax_bind for the numbering), with index = -1 the AoS buffer, with
 * index = -2 the AoSoA buffer (NULL when none is bound). */
soax_status soax_buffer(const soax_set* set, int32_t index, void** ptr);

/*
 * Seeded synthetic fill of every SoA array (SplitMix64, Steele-Lea-Flood
 * 2014, one counter-based stream per field component; Box-Muller normals):
 *   id -> i; tag -> raw draw; pos -> U[0, 2pi); vel, acc -> N(0,1);
 *   mass -> U[0.5, 2); flags -> top 8 bits of a draw; other floats -> U[0,1);
 *   other integers -> low bytes of a draw.
 * vel_mode 1 instead sets vel = u(pos) with params' amplitudes.  The AoS
 * copy is not touched (use soax_soa_to_aos).  Errors: ARG, LAYOUT (no SoA).
 */
soax_status soax_fill(soax_set* set, uint64_t seed, int32_t vel_mode, const soax_params* params,
                      void* stream);

/*
 * nsteps time steps of `integrator` on one layout: SOAX_SOA (vector loads
 * per array), SOAX_AOS (records staged through LDS with coalesced 16-byte
 * accesses), SOAX_AOS_NAIVE (one thread per record, direct per-field
 * accesses, the uncoalesced pattern of Section 3.2), SOAX_AOSOA (the tiled
 * copy, one thread per particle).  Only pos/vel are
 * written; every other byte keeps its value.  params may be NULL for Euler
 * steps without wrap.  Errors: ARG, SCHEMA, LAYOUT, HIP.
 */
soax_status soax_step(soax_set* set, int32_t layout, int32_t integrator, double dt, int64_t nsteps,
                      const soax_params* params, void* stream);

/*
 * nsteps time steps of `integrator` on the SoA arrays in one launch, each
 * particle held in registers from the first step to the last, so the arrays
 * are read and written once per call instead of once per step.  This is not
 * the loop the paper benchmarks (Section 2 passes over every array at each
 * step, which is what soax_step does); it is offered beside it for callers
 * that need nothing between the steps.  Every step is the same arithmetic as
 * soax_step's, so the results equal soax_step(set, SOAX_SOA, integrator, dt,
 * nsteps, params, stream) bit for bit; for the field integrators the
 * velocity (which no step reads) is evaluated once, at the final position.
 * One thread per particle, 256-thread workgroups.  Arguments and errors as
 * soax_step; a single launch runs every step, so its duration grows with
 * nsteps.
 */
soax_status soax_step_fused(soax_set* set, int32_t integrator, double dt, int64_t nsteps,
                            const soax_params* params, void* stream);

/*
 * Override the launch shape of soax_step for one layout: block threads
 * (64..1024, multiple of 64) and particles per thread (1, 2 or 4; SoA only).
 * 0 restores the default: 128 threads (256 for the AoS layouts) and one
 * particle per thread; for the steps in the ABC field (RK2, Heun, RK4) on SoA
 * arrays that are 16-byte aligned and span at least 128 MB (positions and
 * velocities), 64 threads and two particles per thread.
 * Heun and RK4 steps, and any step whose positions or velocities are 8-byte
 * elements, take at most two per thread.  Results do not depend on the
 * shape.
 */
soax_status soax_step_config(soax_set* set, int32_t layout, int32_t block, int32_t per_thread);

/*
 * The nsteps launches of one soax_step call captured once into a hipGraph and
 * replayed by soax_step_graph_launch with a single graph launch: the same
 * results as soax_step with the same arguments, with less launch overhead for
 * sets small enough to be launch-bound.  The buffers, n, dt and params are
 * fixed at capture; a launch after the set changed size or buffers fails with
 * STATE.  Create validates like soax_step (errors ARG, SCHEMA, LAYOUT) and
 * synchronises nothing; the graph must be destroyed before the set.
 */
typedef struct soax_step_graph soax_step_graph;
soax_status soax_step_graph_create(soax_set* set, int32_t layout, int32_t integrator, double dt,
                                   int64_t nsteps, const soax_params* params,
                                   soax_step_graph** out);
soax_status soax_step_graph_launch(soax_step_graph* graph, void* stream);
void soax_step_graph_destroy(soax_step_graph* graph);

/* Bulk transposes between the two copies, byte-exact; soax_soa_to_aos
 * writes every padding byte of every record as 0.  Both need both copies. */
soax_status soax_aos_to_soa(soax_set* set, void* stream);
soax_status soax_soa_to_aos(soax_set* set, void* stream);

/* Copy record i of one layout (SOAX_SOA, SOAX_AOS or SOAX_AOSOA) to host
 * memory in AoS form (stride bytes, padding 0): the particle extracted as one
 * object of all its properties, as the element access of Section 4.1 does.
 * Errors: ARG (null set or record, i outside [0, n), unknown layout),
 * LAYOUT (the set holds no copy in that layout), HIP.  Synchronises the null
 * stream. */
soax_status soax_get_record(const soax_set* set, int32_t layout, int64_t i, void* host_record);

/* ----------------------------------------------------------- AoSoA tiles */

/*
 * An optional third copy in a tiled layout (array of structures of arrays):
 * particles in tiles of 64 (one wavefront); a tile holds, for every SoA array
 * in order, its 64 elements back to back, so element i of array a is at byte
 *   (i / 64) * tile_bytes + array_offsets[a] + (i % 64) * element_size(a),
 * array_offsets[a] = 64 * (element sizes of the arrays before a), tile_bytes
 * = 64 * (sum of all element sizes).  The layout keeps a particle's fields in
 * one few-KB block (like an AoS record) while a wavefront still reads each
 * field as one contiguous run (like SoA).  Not a layout of the paper's
 * benchmark; a variant for comparison.
 */

/* Host only: the tile layout of a schema (array_offsets[narrays] may be NULL). */
soax_status soax_aosoa_layout(const soax_schema* schema, int64_t* array_offsets,
                              int64_t* tile_bytes);

/* Attach a caller-owned, 16-byte aligned buffer of at least
 * ceil(capacity / 64) * tile_bytes bytes as the set's AoSoA copy (NULL
 * detaches); needs the SoA copy.  Contents are undefined until converted.
 * Container calls do not update the AoSoA copy; growth past the capacity and
 * soax_rebind detach it.  Errors: ARG (too small), LAYOUT, OOM, HIP. */
soax_status soax_bind_aosoa(soax_set* set, void* aosoa, int64_t bytes);

/* Conversions between the SoA and AoSoA copies, byte-exact; soa -> aosoa
 * writes the unused lanes of the last tile as zero bytes. */
soax_status soax_soa_to_aosoa(soax_set* set, void* stream);
soax_status soax_aosoa_to_soa(soax_set* set, void* stream);

/* ------------------------------------------------------------ containers */

/*
 * Container operations (the container interface of Section 4.1: resize,
 * element access, push_back; removal of Section 2).  They apply to every copy
 * the set has (SoA and AoS), keep each particle's bytes unchanged and leave
 * the two copies consistent if they were.  A set that changes its size or
 * buffers (any call below but soax_capacity and soax_set_record) invalidates
 * every batch that holds it: such a batch's calls then fail with STATE.
 * Growing past the capacity, push_back and rebind synchronise `stream`
 * before returning; removal waits once for its flag count (the new size is
 * returned) and leaves the moves enqueued; resize within the capacity only
 * enqueues its zero fill.
 */

/* Host query of the particle count and the capacity. */
soax_status soax_capacity(const soax_set* set, int64_t* n, int64_t* capacity);

/* Room for `capacity` particles.  Owned sets (soax_create) move to larger
 * buffers, copying their n particles; bound sets fail with STATE beyond the
 * capacity they were bound with.  Never shrinks.  Errors: ARG, RANGE, STATE,
 * OOM, HIP. */
soax_status soax_reserve(soax_set* set, int64_t capacity, void* stream);

/* New particle count n.  Particles [old n, n) are zero bytes in every copy;
 * shrinking drops the tail.  Owned sets grow to max(n, 2 * capacity) when
 * needed.  Errors: ARG, RANGE, STATE (bound set beyond its capacity), OOM, HIP. */
soax_status soax_resize(soax_set* set, int64_t n, void* stream);

/* Append `count` records given in AoS form in host memory (count * stride
 * bytes, the set's schema and packing): the AoS copy receives the bytes as
 * they are, the SoA copy each field component.  Grows like soax_resize.
 * The host buffer may be reused when the call returns. */
soax_status soax_push_back(soax_set* set, const void* host_records, int64_t count, void* stream);

/* Move a bound set to caller buffers with room for `capacity` >= n
 * particles (the same copies as before: soa_ptrs NULL iff the set has no SoA
 * copy, aos_ptr NULL iff it has no AoS copy), copying its n particles; the
 * old buffers may be freed when the call returns.  Owned sets fail with
 * STATE.  Errors: ARG, RANGE, LAYOUT, STATE, HIP. */
soax_status soax_rebind(soax_set* set, int64_t capacity, void* const* soa_ptrs, void* aos_ptr,
                        void* stream);

/* Write record i (0 <= i < n) of every copy from one AoS-form host record.
 * Synchronous (null stream). */
soax_status soax_set_record(soax_set* set, int64_t i, const void* host_record);

/*
 * Remove every particle i < n with flags[i] != 0 (device, n bytes; not
 * modified; it may be reused once the stream has passed this call) by
 * overwriting it with the last particle, the removal of
 * Section 2 for sets whose order does not matter.  The result equals the
 * sequential rule "while particle i is flagged, copy the last particle over
 * it and drop the last", computed as: the flagged slots below n' = n - m
 * (m flagged particles) in ascending order receive the unflagged particles
 * at or above n' in descending order.  Writes n' to *new_n (host).
 * Errors: ARG, HIP, OOM.
 */
soax_status soax_remove_flagged(soax_set* set, const uint8_t* flags, int64_t* new_n, void* stream);

/* ----------------------------------------------------------- expressions */

/*
 * Fused element-wise expressions over whole arrays (the array access of
 * Section 4.1, e.g. posArr(0) = velArr(1) - velArr(2), and its evaluation as
 * one loop by expression templates, Section 4.2).  A program is a postfix
 * list of ops on a value stack:
 *   SOAX_OP_ARRAY  push element i of array `arg`;   SOAX_OP_CONST  push `value`;
 *   SOAX_OP_ADD, _SUB, _MUL, _DIV  pop b, pop a, push a op b;
 *   SOAX_OP_MIN, _MAX  pop b, pop a, push (a < b ? a : b) / (a > b ? a : b);
 *   SOAX_OP_NEG, _ABS, _SQRT  replace the top value.
 * Every value is a double: array elements are converted to double (exact for
 * every type but i64 beyond 2^53, which rounds to nearest), each operation is
 * one IEEE double operation rounded to nearest (none is fused into an fma),
 * and the result is rounded once to the destination type (f32 or f64).  At
 * most 64 ops, 8 distinct arrays and 32 constants; the stack must end with
 * one value.  The kernel for a program's shape (its ops and element types)
 * is generated and compiled with hipRTC on the first call on a device and
 * cached for the life of the process; constants and pointers are arguments.
 * The destination may also be read by the program (each element is read
 * before it is written).
 */
typedef struct {
  int32_t op;
  int32_t arg;  /* SOAX_OP_ARRAY: array index */
  double value; /* SOAX_OP_CONST: the constant */
} soax_expr_op;
#define SOAX_OP_ARRAY 0
#define SOAX_OP_CONST 1
#define SOAX_OP_ADD 2
#define SOAX_OP_SUB 3
#define SOAX_OP_MUL 4
#define SOAX_OP_DIV 5
#define SOAX_OP_NEG 6
#define SOAX_OP_ABS 7
#define SOAX_OP_SQRT 8
#define SOAX_OP_MIN 9
#define SOAX_OP_MAX 10

/* SoA array dst_array of a set (f32 or f64) = program over the set's SoA
 * arrays (arg = array index, numbered as in soax_bind), for its n particles.
 * Errors: ARG (bad program or index), SCHEMA (integer destination), LAYOUT
 * (no SoA copy), HIP (compilation or launch; the message has the compiler
 * log). */
soax_status soax_eval(soax_set* set, int32_t dst_array, const soax_expr_op* prog, int32_t nops,
                      void* stream);

/* The same over plain device arrays of n elements: src[j] has type
 * src_dtypes[j] (a soax_dtype), arg = j; dst has type dst_dtype (f32 or
 * f64).  Pointers must be aligned to their element size. */
soax_status soax_eval_ptrs(int64_t n, void* dst, int32_t dst_dtype, const void* const* src,
                           const int32_t* src_dtypes, int32_t nsrc, const soax_expr_op* prog,
                           int32_t nops, void* stream);

/* Host only: the HIP source of the kernel a program compiles to, as a
 * NUL-terminated string in buf (size bytes).  Errors: ARG (bad program or
 * buffer too small), SCHEMA. */
soax_status soax_expr_source(const soax_expr_op* prog, int32_t nops, int32_t dst_dtype,
                             const int32_t* src_dtypes, int32_t nsrc, char* buf, int64_t size);

/* ------------------------------------------------ differentiable advection */

/*
 * RK2 (explicit midpoint) advection of n positions in the ABC field with
 * amplitudes abc[3] (host), no wrap: x0[d], xT[d] are device arrays of n
 * doubles (d = 0, 1, 2; xT may alias x0).  The checkpoints of the adjoint,
 * the states before steps 0, k, 2k, ... < nsteps, are written to
 * tape[c][r][i] (device, ceil(nsteps/k) * 9 * n doubles): rows r = 0..2 the
 * position, rows 3..8 sin x, cos x, sin y, cos y, sin z, cos z as the
 * forward evaluated them.  When |dt| (|A| + |B| + |C|) <= 1/64 every step's
 * sines and cosines come from the previous step's by angle addition, with a
 * full evaluation every 20 steps; the results depend on the step index only,
 * never on k.  Errors: ARG (NULL array or tape, n < 0, nsteps < 0, k < 1,
 * non-finite dt or amplitude), RANGE (n > 2^31-1), HIP.
 */
soax_status soax_rk2_forward_ckpt(const double* const* x0, double* const* xT, int64_t n,
                                  const double* abc, double dt, int64_t nsteps, int64_t k,
                                  double* tape, void* stream);

/*
 * Discrete adjoint of soax_rk2_forward_ckpt.  Given lamT[d] = dL/dxT (device),
 * recomputes each k-step segment from its checkpoint and sweeps it backwards
 * (midpoint-rule transpose: mu = dt J(xm)^T lam; lam += mu + dt/2 J(x)^T mu),
 * writing grad_x0[d] = dL/dx0 (device, may alias lamT) and grad_abc[3] =
 * dL/d(A,B,C) (device) summed over particles in a fixed order, so the result
 * is deterministic and independent of k.
 */
soax_status soax_adjoint(const double* tape, const double* const* lamT, int64_t n,
                         const double* abc, double dt, int64_t nsteps, int64_t k,
                         double* const* grad_x0, double* grad_abc, void* stream);

/*
 * soax_adjoint for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, bit for bit, but the per-workgroup
 * partial sums of dL/d(A,B,C) live in a fixed device array of 1 MiB that the
 * library holds on every GPU it runs on until the process ends (its address
 * is looked up once per device, on the first call there).  The call
 * allocates nothing; the caller still provides every input and output.
 * n may be at most SOAX_ADJOINT_NOALLOC_MAX_N (one partial of three doubles
 * per 256 particles); larger n fails with SOAX_E_RANGE before any device
 * call.  Every call on one GPU shares that array: calls that overlap in time
 * on one GPU (different streams, or different host threads) race and give
 * undefined gradients; serialise them, e.g. on one stream.  Errors: ARG,
 * RANGE, STATE (device index beyond 63), HIP.
 */
#define SOAX_ADJOINT_NOALLOC_MAX_N 11184640
soax_status soax_adjoint_noalloc(const double* tape, const double* const* lamT, int64_t n,
                                 const double* abc, double dt, int64_t nsteps, int64_t k,
                                 double* const* grad_x0, double* grad_abc, void* stream);

/* loss = sum_i sum_d (xT - target)^2 into loss[0] (device) and
 * lamT = 2 (xT - target) (device; may be NULL); fixed-order reduction. */
soax_status soax_sqdist_loss(const double* const* xT, const double* const* target, int64_t n,
                             double* const* lamT, double* loss, void* stream);

/* The same three calls with the position-like arrays (x0, xT, lamT,
 * grad_x0) read and written at element i * stride (in doubles, 1..4096):
 * stride 1 is the SoA form above; the record stride / 8 with pointers to a
 * record's pos[d] keeps the positions inside AoS records (the AoS side of
 * the SoA/AoS comparison for the adjoint).  target stays SoA; the tape is
 * always [segment][9][n].  Results are bit-identical to the SoA form. */
soax_status soax_rk2_forward_ckpt_strided(const double* const* x0, double* const* xT, int64_t n,
                                          int64_t stride, const double* abc, double dt,
                                          int64_t nsteps, int64_t k, double* tape, void* stream);
soax_status soax_adjoint_strided(const double* tape, const double* const* lamT, int64_t n,
                                 int64_t stride, const double* abc, double dt, int64_t nsteps,
                                 int64_t k, double* const* grad_x0, double* grad_abc,
                                 void* stream);
soax_status soax_sqdist_loss_strided(const double* const* xT, int64_t stride,
                                     const double* const* target, int64_t n, double* const* lamT,
                                     double* loss, void* stream);

/* --------------------------------------------------------------- batching */

/*
 * A batch of particle sets of one schema (pos f64, vel f32 or f64), stepped
 * together by RK2 in the ABC field with per-set dt and amplitudes.  The sets
 * stay owned by the caller and must outlive the batch.
 */
soax_status soax_batch_create(soax_set* const* sets, int32_t nsets, soax_batch** out);
void soax_batch_destroy(soax_batch* batch);

/*
 * nsteps RK2 steps of every set (wrap on): dt[nsets] and abc[nsets*3] are host arrays.
 * mode 0: one kernel launch per set per step;
 * mode 1: one persistent launch per step covering every set;
 * mode 2: the nsteps persistent launches captured once into a hipGraph
 *         (cached per nsteps and stream) and replayed with one graph launch.
 * All modes give bit-identical results.
 */
soax_status soax_batch_step(soax_batch* batch, const double* dt, const double* abc, int64_t nsteps,
                            int32_t mode, void* stream);

/* Set the batch kernel's shape: block threads (64..512, multiple of 64),
 * particles per thread (1, 2 or 4) and workgroups per CU (1..65536); 0 keeps
 * the current value.  The grid is min(CUs x blocks_per_cu, tiles) workgroups
 * walking the tile list with a grid stride, so a value of at least
 * tiles / CUs gives every tile its own workgroup (the default, with block 256
 * and 1 particle per thread). */
soax_status soax_batch_config(soax_batch* batch, int32_t block, int32_t per_thread,
                              int32_t blocks_per_cu);
soax_status soax_batch_get_config(const soax_batch* batch, int32_t* block, int32_t* per_thread,
                                  int32_t* blocks_per_cu);

/*
 * Autotune the batch kernel's shape by timing candidate shapes on the
 * batch itself (state saved and restored, so particles do not move) and keep
 * the fastest.  Candidates: block 64/128/256/512, particles per thread 1/2,
 * workgroups per CU 2/4/8/16/32/64 and 65536 (one tile per workgroup); the
 * four fastest and the shape in use are timed again with longer runs before
 * the choice.  The runs use the dt and amplitudes of the most recent
 * soax_batch_step (dt = 1e-3, A = B = C = 1 before the first).  If cache_path is not NULL the choice is looked up in / added
 * to that JSON file, keyed by device architecture, set count and particle
 * count.  Synchronises the device.
 */
soax_status soax_batch_tune(soax_batch* batch, const char* cache_path);

/* ------------------------------------------------------------ utilities */

/* dst[0..bytes) = src[0..bytes) with 16-byte loads/stores (16-byte aligned
 * pointers) through the streaming cache policies of the step kernels: the
 * bandwidth probe the step kernels are measured against. */
soax_status soax_copy(void* dst, const void* src, int64_t bytes, void* stream);

/*
 * Bandwidth probes: the memory accesses of the streaming SoA steps with their
 * arithmetic taken out, on caller-owned device arrays pos[3] (n doubles each)
 * and vel[3] (n floats each), one particle per thread (the RK2 step itself
 * takes two), with the step kernels' buffer windows and cache policies (nt
 * loads, sc0 sc1 nt stores).  They measure what the step kernels' access
 * patterns reach on this memory system, as soax_copy does for plain
 * streaming:
 *   SOAX_PROBE_RK2    read pos, write pos (unchanged) and vel = (float)pos:
 *                     the 60 B per particle of an RK2, Heun or RK4 step;
 *   SOAX_PROBE_EULER  per component read pos and vel, write pos (unchanged
 *                     for finite vel): the 60 B of an Euler step;
 *   SOAX_PROBE_READ   read pos only (24 B; writes nothing, vel may be NULL);
 *   SOAX_PROBE_WRITE  write pos = 0 and vel = 0 (36 B; destroys the values).
 * Errors: ARG (bad pattern, NULL array, n < 0), RANGE (n > 2^31-1), HIP.
 */
#define SOAX_PROBE_RK2 0
#define SOAX_PROBE_EULER 1
#define SOAX_PROBE_READ 2
#define SOAX_PROBE_WRITE 3
soax_status soax_probe(int32_t pattern, double* const* pos, float* const* vel, int64_t n,
                       void* stream);

const char* soax_strerror(soax_status status);
const char* soax_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
