"""Seeded synthetic inputs for the particle-update workloads.

The one module that both the GPU path's tests/benchmark and the CPU oracle
draw inputs from.  It holds no arithmetic of the method: only record
schemas, box size, and seeded numpy draws of initial states with the
distributions of the workloads (numpy's PCG64 generator, not the library's
own counter-based fill, which is tested on its own).

Schemas are lists of ``(name, dtype, dim)``; SoA states are lists of 1-D
numpy arrays, one per (field, component), in schema order.
"""
import math

import numpy as np

# Periodic box edge: the double nearest to 2*pi.
BOX_L = 2.0 * math.pi
_BELOW_L = np.nextafter(BOX_L, 0.0)

# The problem-statement record {int id; double pos[3]; float vel[3]}.
BASE_FIELDS = [("id", "i32", 1), ("pos", "f64", 3), ("vel", "f32", 3)]

# Wide heterogeneous record.
WIDE_FIELDS = [("tag", "i64", 1), ("id", "i32", 1), ("pos", "f64", 3), ("vel", "f32", 3),
               ("acc", "f32", 3), ("mass", "f64", 1), ("flags", "u8", 1)]

_NP = {"i8": np.int8, "u8": np.uint8, "i32": np.int32, "i64": np.int64,
       "f32": np.float32, "f64": np.float64}


def particle_size_fields(size):
    """The benchmark particle of the paper: float x[3], float v[3] and SIZE
    extra floats (stored as fields of at most 3 components)."""
    fields = [("pos", "f32", 3), ("vel", "f32", 3)]
    k = 0
    while size > 0:
        d = min(3, size)
        fields.append((f"temp{k}", "f32", d))
        size -= d
        k += 1
    return fields


def _uniform_box(rng, shape):
    return np.minimum(rng.random(shape) * BOX_L, _BELOW_L)


def random_state(fields, n, seed=0):
    """SoA arrays for any schema: ids 0..n-1, positions U[0,L), velocities
    and accelerations N(0,1), mass U(0.5,2), other floats U[0,1), integers
    uniform over their type."""
    rng = np.random.default_rng(seed)
    out = []
    for name, t, d in fields:
        dt = _NP[t]
        for _ in range(d):
            if name == "id":
                a = np.arange(n, dtype=dt)
            elif name == "pos" and t.startswith("f"):
                a = _uniform_box(rng, n).astype(dt)
                if dt == np.float32:
                    a = np.minimum(a, np.float32(6.2831850))
            elif name in ("vel", "acc") and t.startswith("f"):
                a = rng.standard_normal(n).astype(dt)
            elif name == "mass" and t.startswith("f"):
                a = (0.5 + 1.5 * rng.random(n)).astype(dt)
            elif t.startswith("f"):
                a = rng.random(n).astype(dt)
            else:
                info = np.iinfo(dt)
                a = rng.integers(info.min, info.max, size=n, dtype=dt, endpoint=True)
            out.append(np.ascontiguousarray(a))
    return out


def edge_positions(n, seed=0):
    """Positions (3, n) that crowd the periodic boundary: exact 0, the largest
    double below L, tiny values, values one step away from either edge."""
    rng = np.random.default_rng(seed)
    specials = np.array([0.0, 5e-324, 1e-300, 1e-17, 1e-12, 1e-6, 1e-3,
                         BOX_L - 1e-3, BOX_L - 1e-6, BOX_L - 1e-12, BOX_L - 2e-15,
                         _BELOW_L, np.pi, 0.5 * np.pi])
    x = _uniform_box(rng, (3, n))
    pick = rng.random((3, n)) < 0.5
    x[pick] = rng.choice(specials, size=int(pick.sum()))
    return np.ascontiguousarray(x)


def adjoint_inputs(n, seed=0):
    """Initial positions and targets, both U[0,L)^3, as (3, n) float64."""
    rng = np.random.default_rng(seed)
    x0 = _uniform_box(rng, (3, n))
    target = _uniform_box(rng, (3, n))
    return np.ascontiguousarray(x0), np.ascontiguousarray(target)


def batch_plan(nsets=256, lo=1e3, hi=1e6, seed=0):
    """Set sizes log-uniform in [lo, hi], per-set dt U[1e-4, 1e-2] and
    amplitudes (A, B, C) U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(10.0 ** rng.uniform(np.log10(lo), np.log10(hi), nsets)).astype(np.int64)
    sizes = np.clip(sizes, int(lo), int(hi))
    dts = rng.uniform(1e-4, 1e-2, nsets)
    abc = rng.uniform(0.5, 1.5, (nsets, 3))
    return sizes, dts, abc
