/*
 * soaxref.c -- CPU oracle for the SoA/AoS particle-update hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see soaxref.h).  Written from the paper's
 * statement of the problem, not from any GPU code:
 *
 *  - records and their two storage layouts: Section 1 (Listings 1-3, the
 *    AoS struct and the SoA class), Section 2 (Listing 4, the benchmark
 *    particle) and Section 4.1 (the attribute tuple of the usage listing);
 *  - the Euler advection step x += dt v of Section 2, eq. (1), looped over
 *    all particles once per time step;
 *  - the per-element copy between a record and the arrays (Section 1, the
 *    paragraph after Listing 3; Section 4.1, getElement/push_back), here in
 *    bulk form;
 *  - RK2 advection in the ABC field and its discrete adjoint; the paper only
 *    mentions Runge-Kutta schemes as a reason records carry extra temporary
 *    fields (Section 2), so their definitions are the explicit midpoint rule
 *    and its exact reverse-mode derivative, written out below.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math (see build.py).
 */
#include "soaxref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The periodic box edge: the double nearest to 2*pi. */
static const double REF_L = 6.283185307179586;

int soaxref_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* ------------------------------------------------------------------ schema */

static int64_t esize(int32_t dt) {
  switch (dt) {
    case REF_I8: case REF_U8: return 1;
    case REF_I32: case REF_F32: return 4;
    case REF_I64: case REF_F64: return 8;
    default: return 0;
  }
}

static int check_schema(const ref_schema* s) {
  if (!s || s->nfields < 1 || !s->dtypes || !s->dims || !s->names) return -1;
  for (int f = 0; f < s->nfields; ++f) {
    if (esize(s->dtypes[f]) == 0) return -2;
    if (s->dims[f] < 1 || s->dims[f] > 3) return -2;
    if (!s->names[f]) return -2;
  }
  return 0;
}

/*
 * A C struct lays its members out in declaration order; each member starts
 * at the next multiple of its own alignment (for these scalar types, their
 * size) and the struct size is rounded up to the largest member alignment,
 * so that consecutive records in an array stay aligned.  Packed: no padding.
 */
int soaxref_layout(const ref_schema* s, int64_t* offsets, int64_t* stride) {
  int rc = check_schema(s);
  if (rc) return rc;
  int64_t end = 0, maxal = 1;
  for (int f = 0; f < s->nfields; ++f) {
    int64_t es = esize(s->dtypes[f]);
    if (!s->packed && end % es) end += es - end % es;
    if (offsets) offsets[f] = end;
    end += es * s->dims[f];
    if (es > maxal) maxal = es;
  }
  if (!s->packed && end % maxal) end += maxal - end % maxal;
  if (stride) *stride = end;
  return 0;
}

static int find_field(const ref_schema* s, const char* name) {
  for (int f = 0; f < s->nfields; ++f)
    if (strcmp(s->names[f], name) == 0) return f;
  return -1;
}

/* index of the first SoA array of field f */
static int first_array(const ref_schema* s, int f) {
  int a = 0;
  for (int g = 0; g < f; ++g) a += s->dims[g];
  return a;
}

/* ----------------------------------------------------------- element views */

/* Component c of particle i of a 3-vector field sits at base[c] + i*step. */
typedef struct {
  char* base[3];
  int64_t step;
  int32_t dtype;
} vec_view;

static double vload(const vec_view* v, int64_t i, int c) {
  const char* p = v->base[c] + i * v->step;
  if (v->dtype == REF_F64) {
    double x;
    memcpy(&x, p, 8);
    return x;
  }
  float x;
  memcpy(&x, p, 4);
  return (double)x;
}

static void vstore(const vec_view* v, int64_t i, int c, double x) {
  char* p = v->base[c] + i * v->step;
  if (v->dtype == REF_F64) {
    memcpy(p, &x, 8);
  } else {
    float y = (float)x;
    memcpy(p, &y, 4);
  }
}

static int is_float(int32_t dt) { return dt == REF_F32 || dt == REF_F64; }

static int soa_view(const ref_schema* s, void* const* soa, const char* name, vec_view* v) {
  int f = find_field(s, name);
  if (f < 0 || s->dims[f] != 3 || !is_float(s->dtypes[f])) return -2;
  int a = first_array(s, f);
  for (int c = 0; c < 3; ++c) {
    if (!soa[a + c]) return -1;
    v->base[c] = (char*)soa[a + c];
  }
  v->step = esize(s->dtypes[f]);
  v->dtype = s->dtypes[f];
  return 0;
}

static int aos_view(const ref_schema* s, void* aos, const char* name, vec_view* v) {
  int64_t off[64], stride;
  if (s->nfields > 64) return -2;
  soaxref_layout(s, off, &stride);
  int f = find_field(s, name);
  if (f < 0 || s->dims[f] != 3 || !is_float(s->dtypes[f])) return -2;
  int64_t es = esize(s->dtypes[f]);
  for (int c = 0; c < 3; ++c) v->base[c] = (char*)aos + off[f] + c * es;
  v->step = stride;
  v->dtype = s->dtypes[f];
  return 0;
}

/* ------------------------------------------------------------------- maths */

/* Periodic wrap of a coordinate displaced by much less than one box edge. */
static double wrap_box(double x) {
  if (x >= REF_L) {
    x -= REF_L;
  } else if (x < 0.0) {
    x += REF_L;
    if (x >= REF_L) x = 0.0; /* a tiny negative x whose sum rounds up to L */
  }
  return x;
}

/* ABC (Arnold-Beltrami-Childress) flow with amplitudes (A, B, C):
 * u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x). */
void soaxref_field(const double* abc, const double* x, double* u) {
  const double A = abc[0], B = abc[1], C = abc[2];
  u[0] = A * sin(x[2]) + C * cos(x[1]);
  u[1] = B * sin(x[0]) + A * cos(x[2]);
  u[2] = C * sin(x[1]) + B * cos(x[0]);
}

/* One explicit-midpoint step: k1 = u(x), xm = x + (dt/2) k1, x+ = x + dt u(xm). */
static void rk2_midpoint(const double* abc, double dt, const double* x, double* xn) {
  double k1[3], xm[3], k2[3];
  soaxref_field(abc, x, k1);
  for (int d = 0; d < 3; ++d) xm[d] = x[d] + (0.5 * dt) * k1[d];
  soaxref_field(abc, xm, k2);
  for (int d = 0; d < 3; ++d) xn[d] = x[d] + dt * k2[d];
}

/* One Heun (explicit trapezoidal) step: k1 = u(x), k2 = u(x + dt k1),
 * x+ = x + (dt/2)(k1 + k2). */
static void heun(const double* abc, double dt, const double* x, double* xn) {
  double k1[3], xp[3], k2[3];
  soaxref_field(abc, x, k1);
  for (int d = 0; d < 3; ++d) xp[d] = x[d] + dt * k1[d];
  soaxref_field(abc, xp, k2);
  for (int d = 0; d < 3; ++d) xn[d] = x[d] + (0.5 * dt) * (k1[d] + k2[d]);
}

/* One classical fourth-order Runge-Kutta step: k1 = u(x), k2 = u(x + dt/2 k1),
 * k3 = u(x + dt/2 k2), k4 = u(x + dt k3), x+ = x + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
static void rk4(const double* abc, double dt, const double* x, double* xn) {
  double k1[3], k2[3], k3[3], k4[3], y[3];
  soaxref_field(abc, x, k1);
  for (int d = 0; d < 3; ++d) y[d] = x[d] + (0.5 * dt) * k1[d];
  soaxref_field(abc, y, k2);
  for (int d = 0; d < 3; ++d) y[d] = x[d] + (0.5 * dt) * k2[d];
  soaxref_field(abc, y, k3);
  for (int d = 0; d < 3; ++d) y[d] = x[d] + dt * k3[d];
  soaxref_field(abc, y, k4);
  for (int d = 0; d < 3; ++d)
    xn[d] = x[d] + (dt / 6.0) * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
}

static int field_integrator(int integ) {
  return integ == REF_RK2_ABC || integ == REF_HEUN_ABC || integ == REF_RK4_ABC;
}

/* Advance particle i by one step of the chosen integrator. */
static void particle_step(int integ, const vec_view* P, const vec_view* V, const vec_view* Acc,
                          int64_t i, double dt, const double* abc, int wrap) {
  double x[3];
  for (int d = 0; d < 3; ++d) x[d] = vload(P, i, d);
  if (integ == REF_EULER || integ == REF_EULER_ACC) {
    /* eq. (1): x += dt v, per component, with the velocity before any update */
    for (int d = 0; d < 3; ++d) {
      double v = vload(V, i, d);
      double xn = x[d] + dt * v;
      if (wrap) xn = wrap_box(xn);
      vstore(P, i, d, xn);
      if (integ == REF_EULER_ACC) {
        double a = vload(Acc, i, d);
        vstore(V, i, d, v + dt * a);
      }
    }
  } else if (integ == REF_SYMPLECTIC_EULER) {
    /* the velocity first (stored in its own type), then the position with
     * the new velocity */
    for (int d = 0; d < 3; ++d) {
      vstore(V, i, d, vload(V, i, d) + dt * vload(Acc, i, d));
      double xn = x[d] + dt * vload(V, i, d);
      if (wrap) xn = wrap_box(xn);
      vstore(P, i, d, xn);
    }
  } else {
    double xn[3], un[3];
    if (integ == REF_RK2_ABC)
      rk2_midpoint(abc, dt, x, xn);
    else if (integ == REF_HEUN_ABC)
      heun(abc, dt, x, xn);
    else
      rk4(abc, dt, x, xn);
    if (wrap)
      for (int d = 0; d < 3; ++d) xn[d] = wrap_box(xn[d]);
    for (int d = 0; d < 3; ++d) vstore(P, i, d, xn[d]);
    soaxref_field(abc, xn, un); /* the stored velocity is the field at the new position */
    for (int d = 0; d < 3; ++d) vstore(V, i, d, un[d]);
  }
}

static int check_step_args(const ref_schema* s, int64_t n, int integ, double dt, int64_t nsteps,
                           const double* abc, int wrap) {
  if (n < 0 || nsteps < 0 || !isfinite(dt)) return -1;
  if (integ < REF_EULER || integ > REF_SYMPLECTIC_EULER) return -1;
  if (field_integrator(integ)) {
    if (!abc || !isfinite(abc[0]) || !isfinite(abc[1]) || !isfinite(abc[2])) return -1;
    int f = find_field(s, "pos");
    if (f < 0 || s->dtypes[f] != REF_F64) return -2;
  }
  if (wrap) {
    int f = find_field(s, "pos");
    if (f < 0 || s->dtypes[f] != REF_F64) return -2;
  }
  return 0;
}

static int run_steps(const ref_schema* s, int64_t n, const vec_view* P, const vec_view* V,
                     const vec_view* Acc, int integ, double dt, int64_t nsteps, const double* abc,
                     int wrap) {
  /* one full sweep over all particles per time step (Section 2) */
  for (int64_t t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) particle_step(integ, P, V, Acc, i, dt, abc, wrap);
  }
  (void)s;
  return 0;
}

int soaxref_step_soa(const ref_schema* s, int64_t n, void* const* soa, int integ, double dt,
                     int64_t nsteps, const double* abc, int wrap) {
  int rc = check_schema(s);
  if (rc) return rc;
  if (!soa) return -1;
  if ((rc = check_step_args(s, n, integ, dt, nsteps, abc, wrap))) return rc;
  vec_view P, V, Acc;
  if ((rc = soa_view(s, soa, "pos", &P))) return rc;
  if ((rc = soa_view(s, soa, "vel", &V))) return rc;
  if ((integ == REF_EULER_ACC || integ == REF_SYMPLECTIC_EULER) &&
      (rc = soa_view(s, soa, "acc", &Acc)))
    return rc;
  return run_steps(s, n, &P, &V, &Acc, integ, dt, nsteps, abc, wrap);
}

int soaxref_step_aos(const ref_schema* s, int64_t n, void* aos, int integ, double dt,
                     int64_t nsteps, const double* abc, int wrap) {
  int rc = check_schema(s);
  if (rc) return rc;
  if (!aos && n > 0) return -1;
  if ((rc = check_step_args(s, n, integ, dt, nsteps, abc, wrap))) return rc;
  vec_view P, V, Acc;
  if ((rc = aos_view(s, aos, "pos", &P))) return rc;
  if ((rc = aos_view(s, aos, "vel", &V))) return rc;
  if ((integ == REF_EULER_ACC || integ == REF_SYMPLECTIC_EULER) &&
      (rc = aos_view(s, aos, "acc", &Acc)))
    return rc;
  return run_steps(s, n, &P, &V, &Acc, integ, dt, nsteps, abc, wrap);
}

/* -------------------------------------------------------------- transposes */

int soaxref_aos_to_soa(const ref_schema* s, int64_t n, const void* aos, void* const* soa) {
  int64_t off[64], stride;
  int rc = check_schema(s);
  if (rc) return rc;
  if (s->nfields > 64 || n < 0 || !soa || (!aos && n > 0)) return -1;
  soaxref_layout(s, off, &stride);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int f = 0; f < s->nfields; ++f) {
      int64_t es = esize(s->dtypes[f]);
      int a = first_array(s, f);
      for (int c = 0; c < s->dims[f]; ++c)
        memcpy((char*)soa[a + c] + i * es, (const char*)aos + i * stride + off[f] + c * es, es);
    }
  }
  return 0;
}

int soaxref_soa_to_aos(const ref_schema* s, int64_t n, void* const* soa, void* aos) {
  int64_t off[64], stride;
  int rc = check_schema(s);
  if (rc) return rc;
  if (s->nfields > 64 || n < 0 || !soa || (!aos && n > 0)) return -1;
  soaxref_layout(s, off, &stride);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    char* rec = (char*)aos + i * stride;
    memset(rec, 0, stride);
    for (int f = 0; f < s->nfields; ++f) {
      int64_t es = esize(s->dtypes[f]);
      int a = first_array(s, f);
      for (int c = 0; c < s->dims[f]; ++c)
        memcpy(rec + off[f] + c * es, (const char*)soa[a + c] + i * es, es);
    }
  }
  return 0;
}

/* -------------------------------------------------------------- AoSoA tiles */

int soaxref_aosoa_layout(const ref_schema* s, int64_t* array_offsets, int64_t* tile_bytes) {
  int rc = check_schema(s);
  if (rc) return rc;
  int64_t acc = 0;
  for (int f = 0; f < s->nfields; ++f) {
    int a = first_array(s, f);
    for (int c = 0; c < s->dims[f]; ++c) {
      if (array_offsets) array_offsets[a + c] = REF_AOSOA_W * acc;
      acc += esize(s->dtypes[f]);
    }
  }
  if (tile_bytes) *tile_bytes = REF_AOSOA_W * acc;
  return 0;
}

int soaxref_soa_to_aosoa(const ref_schema* s, int64_t n, void* const* soa, void* aosoa) {
  int64_t aoff[3 * 64], tile;
  int rc = check_schema(s);
  if (rc) return rc;
  if (n < 0 || !soa || (!aosoa && n > 0)) return -1;
  soaxref_aosoa_layout(s, aoff, &tile);
  const int64_t ntiles = (n + REF_AOSOA_W - 1) / REF_AOSOA_W;
  memset(aosoa, 0, (size_t)(ntiles * tile));
  for (int64_t i = 0; i < n; ++i) {
    char* t = (char*)aosoa + (i / REF_AOSOA_W) * tile;
    for (int f = 0; f < s->nfields; ++f) {
      int64_t es = esize(s->dtypes[f]);
      int a = first_array(s, f);
      for (int c = 0; c < s->dims[f]; ++c)
        memcpy(t + aoff[a + c] + (i % REF_AOSOA_W) * es, (const char*)soa[a + c] + i * es, es);
    }
  }
  return 0;
}

int soaxref_aosoa_to_soa(const ref_schema* s, int64_t n, const void* aosoa, void* const* soa) {
  int64_t aoff[3 * 64], tile;
  int rc = check_schema(s);
  if (rc) return rc;
  if (n < 0 || !soa || (!aosoa && n > 0)) return -1;
  soaxref_aosoa_layout(s, aoff, &tile);
  for (int64_t i = 0; i < n; ++i) {
    const char* t = (const char*)aosoa + (i / REF_AOSOA_W) * tile;
    for (int f = 0; f < s->nfields; ++f) {
      int64_t es = esize(s->dtypes[f]);
      int a = first_array(s, f);
      for (int c = 0; c < s->dims[f]; ++c)
        memcpy((char*)soa[a + c] + i * es, t + aoff[a + c] + (i % REF_AOSOA_W) * es, es);
    }
  }
  return 0;
}

/* ------------------------------------------------------------- containers */

/*
 * Removal without keeping the order (Section 2, the paragraph on std::vector
 * vs std::list: a particle is removed by overwriting it with the last
 * particle).  Sequentially, for i = 0, 1, ...: while particle i is flagged and
 * i < n, copy particle n-1 (and its flag) over it and shrink n by one.
 * flags[] is updated alongside; returns the new count.
 */
int64_t soaxref_remove_flagged(const ref_schema* s, int64_t n, void* const* soa, uint8_t* flags) {
  if (check_schema(s) || n < 0 || !soa || (!flags && n > 0)) return -1;
  int64_t i = 0;
  while (i < n) {
    if (!flags[i]) {
      ++i;
      continue;
    }
    const int64_t last = n - 1;
    if (last != i) {
      for (int f = 0; f < s->nfields; ++f) {
        int64_t es = esize(s->dtypes[f]);
        int a = first_array(s, f);
        for (int c = 0; c < s->dims[f]; ++c)
          memcpy((char*)soa[a + c] + i * es, (const char*)soa[a + c] + last * es, es);
      }
      flags[i] = flags[last];
    }
    n = last;
  }
  return n;
}

/* -------------------------------------------------------------------- fill */

static const uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ULL;

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t soaxref_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Draw i of stream s: the i-th SplitMix64 output from a generator whose seed
 * is the s-th SplitMix64 output from `seed`. */
uint64_t soaxref_draw(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t key = soaxref_mix64(seed + GOLDEN_GAMMA * (stream + 1));
  return soaxref_mix64(key + GOLDEN_GAMMA * (i + 1));
}

static double unit_open1(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }        /* [0,1) */
static double unit_open0(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }  /* (0,1] */

/* Box-Muller: one standard normal from two uniforms. */
static double std_normal(uint64_t seed, uint64_t s, uint64_t i) {
  double u1 = unit_open0(soaxref_draw(seed, s, i));
  double u2 = unit_open1(soaxref_draw(seed, s + 1, i));
  return sqrt(-2.0 * log(u1)) * cos(REF_L * u2);
}

static void store_int(char* p, int32_t dt, uint64_t v) {
  switch (dt) {
    case REF_I8: case REF_U8: { uint8_t x = (uint8_t)v; memcpy(p, &x, 1); break; }
    case REF_I32: { uint32_t x = (uint32_t)v; memcpy(p, &x, 4); break; }
    case REF_I64: memcpy(p, &v, 8); break;
    default: break;
  }
}

static void store_real(char* p, int32_t dt, double v) {
  if (dt == REF_F64) {
    memcpy(p, &v, 8);
  } else {
    float x = (float)v;
    memcpy(p, &x, 4);
  }
}

/*
 * Field rules, by name (streams are 8*f + 2*c [+1] for field f, component c):
 *   id    : i                      tag   : the raw 64-bit draw
 *   pos   : L * U[0,1)             mass  : 0.5 + 1.5 * U[0,1)
 *   vel   : N(0,1) (vel_mode 0) or the field u(pos) (vel_mode 1)
 *   acc   : N(0,1)                 flags : top 8 bits of the draw
 *   other : float -> U[0,1); integer -> low bytes of the draw
 */
int soaxref_fill(const ref_schema* s, int64_t n, uint64_t seed, int vel_mode, const double* abc,
                 void* const* soa) {
  return soaxref_fill_range(s, 0, n, seed, vel_mode, abc, soa);
}

int soaxref_fill_range(const ref_schema* s, int64_t first, int64_t n, uint64_t seed, int vel_mode,
                       const double* abc, void* const* soa) {
  int rc = check_schema(s);
  if (rc) return rc;
  if (n < 0 || first < 0 || !soa || (vel_mode != 0 && vel_mode != 1)) return -1;
  int fpos = find_field(s, "pos"), fvel = find_field(s, "vel");
  if (vel_mode == 1) {
    if (!abc || fpos < 0 || fvel < 0 || s->dims[fpos] != 3 || s->dims[fvel] != 3) return -2;
    if (!is_float(s->dtypes[fpos]) || !is_float(s->dtypes[fvel])) return -2;
  }
  for (int f = 0; f < s->nfields; ++f) {
    const char* nm = s->names[f];
    int32_t dt = s->dtypes[f];
    int64_t es = esize(dt);
    int a = first_array(s, f);
    if (f == fvel && vel_mode == 1) continue; /* after pos, below */
    for (int c = 0; c < s->dims[f]; ++c) {
      char* arr = (char*)soa[a + c];
      uint64_t st = 8 * (uint64_t)f + 2 * (uint64_t)c;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        char* p = arr + i * es;
        const uint64_t gi = (uint64_t)(first + i); /* particle index */
        uint64_t r = soaxref_draw(seed, st, gi);
        if (strcmp(nm, "id") == 0) {
          if (is_float(dt)) store_real(p, dt, (double)gi); else store_int(p, dt, gi);
        } else if (strcmp(nm, "pos") == 0 && is_float(dt)) {
          store_real(p, dt, REF_L * unit_open1(r));
        } else if ((strcmp(nm, "vel") == 0 || strcmp(nm, "acc") == 0) && is_float(dt)) {
          store_real(p, dt, std_normal(seed, st, gi));
        } else if (strcmp(nm, "mass") == 0 && is_float(dt)) {
          store_real(p, dt, 0.5 + 1.5 * unit_open1(r));
        } else if (strcmp(nm, "flags") == 0 && !is_float(dt)) {
          store_int(p, dt, r >> 56);
        } else if (is_float(dt)) {
          store_real(p, dt, unit_open1(r));
        } else {
          store_int(p, dt, r);
        }
      }
    }
  }
  if (vel_mode == 1) {
    vec_view P, V;
    if ((rc = soa_view(s, soa, "pos", &P)) || (rc = soa_view(s, soa, "vel", &V))) return rc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double x[3], u[3];
      for (int d = 0; d < 3; ++d) x[d] = vload(&P, i, d);
      soaxref_field(abc, x, u);
      for (int d = 0; d < 3; ++d) vstore(&V, i, d, u[d]);
    }
  }
  return 0;
}

/* ------------------------------------------------------- RK2 and adjoints */

static int check_abc(const double* abc) {
  return abc && isfinite(abc[0]) && isfinite(abc[1]) && isfinite(abc[2]);
}

int soaxref_rk2_forward(int64_t n, const double* const* x0, double* const* xT, const double* abc,
                        double dt, int64_t nsteps, double* states) {
  if (n < 0 || nsteps < 0 || !isfinite(dt) || !check_abc(abc) || !x0 || !xT) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double x[3], xn[3];
    for (int d = 0; d < 3; ++d) x[d] = x0[d][i];
    if (states)
      for (int d = 0; d < 3; ++d) states[(0 * 3 + d) * n + i] = x[d];
    for (int64_t t = 0; t < nsteps; ++t) {
      rk2_midpoint(abc, dt, x, xn);
      for (int d = 0; d < 3; ++d) x[d] = xn[d];
      if (states)
        for (int d = 0; d < 3; ++d) states[((t + 1) * 3 + d) * n + i] = x[d];
    }
    for (int d = 0; d < 3; ++d) xT[d][i] = x[d];
  }
  return 0;
}

double soaxref_sqdist_loss(int64_t n, const double* const* xT, const double* const* target,
                           double* const* lamT) {
  double loss = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) {
      double e = xT[d][i] - target[d][i];
      loss += e * e;
      if (lamT) lamT[d][i] = 2.0 * e;
    }
  }
  return loss;
}

/* Jacobian of the field, J[r][c] = d u_r / d x_c. */
static void field_jacobian(const double* abc, const double* x, double J[3][3]) {
  const double A = abc[0], B = abc[1], C = abc[2];
  J[0][0] = 0.0;             J[0][1] = -C * sin(x[1]); J[0][2] = A * cos(x[2]);
  J[1][0] = B * cos(x[0]);   J[1][1] = 0.0;            J[1][2] = -A * sin(x[2]);
  J[2][0] = -B * sin(x[0]);  J[2][1] = C * cos(x[1]);  J[2][2] = 0.0;
}

/* Derivative of the field with respect to the amplitudes, G[r][j] = d u_r / d (A,B,C)_j. */
static void field_param_jacobian(const double* x, double G[3][3]) {
  G[0][0] = sin(x[2]); G[0][1] = 0.0;       G[0][2] = cos(x[1]);
  G[1][0] = cos(x[2]); G[1][1] = sin(x[0]); G[1][2] = 0.0;
  G[2][0] = 0.0;       G[2][1] = cos(x[0]); G[2][2] = sin(x[1]);
}

/* out = M^T v */
static void mat_t_vec(double M[3][3], const double* v, double* out) {
  for (int c = 0; c < 3; ++c) out[c] = M[0][c] * v[0] + M[1][c] * v[1] + M[2][c] * v[2];
}

/*
 * Reverse of one midpoint step.  With xm = x + (dt/2) u(x) and
 * x+ = x + dt u(xm):
 *   dx+/dx     = I + dt J(xm) (I + (dt/2) J(x))
 *   dx+/dtheta = dt G(xm) + dt J(xm) (dt/2) G(x)
 * so with mu = dt J(xm)^T lam+ :
 *   lam  = lam+ + mu + (dt/2) J(x)^T mu
 *   g   += dt G(xm)^T lam+ + (dt/2) G(x)^T mu
 */
static void rk2_reverse(const double* abc, double dt, const double* x, double* lam, double* g) {
  double k1[3], xm[3], J[3][3], G[3][3], t[3], mu[3], q[3], r[3];
  soaxref_field(abc, x, k1);
  for (int d = 0; d < 3; ++d) xm[d] = x[d] + (0.5 * dt) * k1[d];
  field_jacobian(abc, xm, J);
  mat_t_vec(J, lam, t);
  for (int d = 0; d < 3; ++d) mu[d] = dt * t[d];
  field_param_jacobian(xm, G);
  mat_t_vec(G, lam, q);
  field_param_jacobian(x, G);
  mat_t_vec(G, mu, r);
  for (int j = 0; j < 3; ++j) g[j] += dt * q[j] + (0.5 * dt) * r[j];
  field_jacobian(abc, x, J);
  mat_t_vec(J, mu, t);
  for (int d = 0; d < 3; ++d) lam[d] = lam[d] + mu[d] + (0.5 * dt) * t[d];
}

int soaxref_adjoint(int64_t n, const double* const* x0, const double* const* lamT,
                    const double* abc, double dt, int64_t nsteps, double* const* grad_x0,
                    double* grad_abc) {
  if (n < 0 || nsteps < 0 || !isfinite(dt) || !check_abc(abc) || !x0 || !lamT || !grad_x0 ||
      !grad_abc)
    return -1;
  double* gpart = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!gpart) return -1;
  int fail = 0;
#pragma omp parallel
  {
    double* xs = (double*)malloc(sizeof(double) * 3 * (size_t)(nsteps + 1));
    if (!xs) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      if (!xs) continue;
      /* store every state x_0..x_{T-1} */
      for (int d = 0; d < 3; ++d) xs[d] = x0[d][i];
      for (int64_t t = 0; t < nsteps; ++t) rk2_midpoint(abc, dt, xs + 3 * t, xs + 3 * (t + 1));
      double lam[3] = {lamT[0][i], lamT[1][i], lamT[2][i]};
      double g[3] = {0.0, 0.0, 0.0};
      for (int64_t t = nsteps - 1; t >= 0; --t) rk2_reverse(abc, dt, xs + 3 * t, lam, g);
      for (int d = 0; d < 3; ++d) grad_x0[d][i] = lam[d];
      for (int j = 0; j < 3; ++j) gpart[3 * i + j] = g[j];
    }
    free(xs);
  }
  if (fail) {
    free(gpart);
    return -1;
  }
  grad_abc[0] = grad_abc[1] = grad_abc[2] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < 3; ++j) grad_abc[j] += gpart[3 * i + j];
  free(gpart);
  return 0;
}

/* C = M + s * (X Y + Z)  (Z may be NULL) */
static void mat_update(double M[3][3], double s, double X[3][3], double Y[3][3], double Z[3][3],
                       double out[3][3]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double xy = X[r][0] * Y[0][c] + X[r][1] * Y[1][c] + X[r][2] * Y[2][c];
      if (Z) xy += Z[r][c];
      out[r][c] = M[r][c] + s * xy;
    }
}

int soaxref_tangent(int64_t n, const double* const* x0, const double* const* lamT,
                    const double* abc, double dt, int64_t nsteps, double* const* grad_x0,
                    double* grad_abc) {
  if (n < 0 || nsteps < 0 || !isfinite(dt) || !check_abc(abc) || !x0 || !lamT || !grad_x0 ||
      !grad_abc)
    return -1;
  double* gpart = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!gpart) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double x[3] = {x0[0][i], x0[1][i], x0[2][i]};
    double M[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}; /* dx/dx0 */
    double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}; /* dx/d(A,B,C) */
    for (int64_t t = 0; t < nsteps; ++t) {
      double k1[3], xm[3], k2[3], J[3][3], G[3][3], Jm[3][3], Gm[3][3];
      double Mm[3][3], Pm[3][3];
      soaxref_field(abc, x, k1);
      field_jacobian(abc, x, J);
      field_param_jacobian(x, G);
      for (int d = 0; d < 3; ++d) xm[d] = x[d] + (0.5 * dt) * k1[d];
      mat_update(M, 0.5 * dt, J, M, NULL, Mm);
      mat_update(P, 0.5 * dt, J, P, G, Pm);
      soaxref_field(abc, xm, k2);
      field_jacobian(abc, xm, Jm);
      field_param_jacobian(xm, Gm);
      for (int d = 0; d < 3; ++d) x[d] = x[d] + dt * k2[d];
      mat_update(M, dt, Jm, Mm, NULL, M);
      mat_update(P, dt, Jm, Pm, Gm, P);
    }
    double lam[3] = {lamT[0][i], lamT[1][i], lamT[2][i]}, gx[3], gp[3];
    mat_t_vec(M, lam, gx);
    mat_t_vec(P, lam, gp);
    for (int d = 0; d < 3; ++d) grad_x0[d][i] = gx[d];
    for (int j = 0; j < 3; ++j) gpart[3 * i + j] = gp[j];
  }
  grad_abc[0] = grad_abc[1] = grad_abc[2] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < 3; ++j) grad_abc[j] += gpart[3 * i + j];
  free(gpart);
  return 0;
}
