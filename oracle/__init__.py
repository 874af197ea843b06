"""CPU oracle for the SoA/AoS particle-update hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never imports, links
or calls anything here, and this package never touches the GPU library.

Thin numpy/ctypes front end over ``libsoaxref.so`` (plain C, fp64, glibc
libm; see soaxref.c for the definition of each routine and the passage of
the paper it follows).

Schemas are lists of ``(name, dtype, dim)`` with dtype one of
``i8 u8 i32 i64 f32 f64``.  SoA data is a list of 1-D numpy arrays, one per
(field, component), in field order then component order.
"""
import ctypes
import os

import numpy as np

from . import build as _build

DTYPES = {"i8": (1, np.int8), "u8": (2, np.uint8), "i32": (3, np.int32),
          "i64": (4, np.int64), "f32": (5, np.float32), "f64": (6, np.float64)}
EULER, EULER_ACC, RK2_ABC, HEUN_ABC, RK4_ABC, SYMPLECTIC_EULER = 0, 1, 2, 3, 4, 5

_lib = None


class _Schema(ctypes.Structure):
    _fields_ = [("nfields", ctypes.c_int32), ("names", ctypes.POINTER(ctypes.c_char_p)),
                ("dtypes", ctypes.POINTER(ctypes.c_int32)), ("dims", ctypes.POINTER(ctypes.c_int32)),
                ("packed", ctypes.c_int32)]


def lib():
    """Load the oracle library, building it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.OUT):
            _build.build()
        L = ctypes.CDLL(_build.OUT)
        vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        sp = ctypes.POINTER(_Schema)
        L.soaxref_threads.argtypes = [i32]
        L.soaxref_layout.argtypes = [sp, vp, vp]
        L.soaxref_mix64.argtypes = [ctypes.c_uint64]
        L.soaxref_mix64.restype = ctypes.c_uint64
        L.soaxref_draw.argtypes = [ctypes.c_uint64] * 3
        L.soaxref_draw.restype = ctypes.c_uint64
        L.soaxref_fill.argtypes = [sp, i64, ctypes.c_uint64, i32, vp, vp]
        L.soaxref_fill_range.argtypes = [sp, i64, i64, ctypes.c_uint64, i32, vp, vp]
        L.soaxref_remove_flagged.argtypes = [sp, i64, vp, vp]
        L.soaxref_remove_flagged.restype = i64
        L.soaxref_field.argtypes = [vp, vp, vp]
        L.soaxref_field.restype = None
        L.soaxref_step_soa.argtypes = [sp, i64, vp, i32, dbl, i64, vp, i32]
        L.soaxref_step_aos.argtypes = [sp, i64, vp, i32, dbl, i64, vp, i32]
        L.soaxref_aos_to_soa.argtypes = [sp, i64, vp, vp]
        L.soaxref_soa_to_aos.argtypes = [sp, i64, vp, vp]
        L.soaxref_aosoa_layout.argtypes = [sp, vp, vp]
        L.soaxref_soa_to_aosoa.argtypes = [sp, i64, vp, vp]
        L.soaxref_aosoa_to_soa.argtypes = [sp, i64, vp, vp]
        L.soaxref_rk2_forward.argtypes = [i64, vp, vp, vp, dbl, i64, vp]
        L.soaxref_sqdist_loss.argtypes = [i64, vp, vp, vp]
        L.soaxref_sqdist_loss.restype = dbl
        L.soaxref_adjoint.argtypes = [i64, vp, vp, vp, dbl, i64, vp, vp]
        L.soaxref_tangent.argtypes = [i64, vp, vp, vp, dbl, i64, vp, vp]
        _lib = L
    return _lib


def threads(n=0):
    """Set the OpenMP thread count if n > 0; return the count in use."""
    return lib().soaxref_threads(int(n))


class Schema:
    """A particle schema as the oracle sees it."""

    def __init__(self, fields, packed=False):
        self.fields = [(str(n), str(t), int(d)) for n, t, d in fields]
        self.packed = bool(packed)
        nf = len(self.fields)
        self._names = (ctypes.c_char_p * nf)(*[f[0].encode() for f in self.fields])
        self._dtypes = (ctypes.c_int32 * nf)(*[DTYPES[f[1]][0] for f in self.fields])
        self._dims = (ctypes.c_int32 * nf)(*[f[2] for f in self.fields])
        self._c = _Schema(nf, self._names, self._dtypes, self._dims, int(self.packed))

    @property
    def ref(self):
        return ctypes.byref(self._c)

    def arrays(self):
        """(field name, component, numpy dtype) of every SoA array, in order."""
        out = []
        for name, t, d in self.fields:
            for c in range(d):
                out.append((name, c, DTYPES[t][1]))
        return out

    def array_index(self, name, comp=0):
        a = 0
        for fname, _, d in self.fields:
            if fname == name:
                return a + comp
            a += d
        raise KeyError(name)

    def layout(self):
        nf = len(self.fields)
        off = (ctypes.c_int64 * nf)()
        stride = ctypes.c_int64()
        rc = lib().soaxref_layout(self.ref, off, ctypes.byref(stride))
        if rc:
            raise ValueError(f"soaxref_layout: {rc}")
        return list(off), stride.value


def _ptrs(arrays):
    for a in arrays:
        assert a.flags["C_CONTIGUOUS"]
    return (ctypes.c_void_p * len(arrays))(*[a.ctypes.data for a in arrays])


def _rows(x):
    """Row pointers of a (3, n) C-contiguous float64 array."""
    assert x.dtype == np.float64 and x.flags["C_CONTIGUOUS"] and x.shape[0] == 3
    return (ctypes.c_void_p * 3)(*[x[d].ctypes.data for d in range(3)])


def _abc(abc):
    a = np.ascontiguousarray(abc if abc is not None else [0.0, 0.0, 0.0], dtype=np.float64)
    return a, a.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def empty_soa(schema, n):
    return [np.zeros(n, dtype=t) for _, _, t in schema.arrays()]


def fill(schema, n, seed=0, vel_mode=0, abc=None):
    arrays = empty_soa(schema, n)
    a, ap = _abc(abc)
    _check(lib().soaxref_fill(schema.ref, n, seed, vel_mode, ap if abc is not None else None,
                              _ptrs(arrays)), "soaxref_fill")
    return arrays


def fill_range(schema, first, count, seed=0, vel_mode=0, abc=None):
    """Fill values of particles first .. first+count-1."""
    arrays = empty_soa(schema, count)
    a, ap = _abc(abc)
    _check(lib().soaxref_fill_range(schema.ref, first, count, seed, vel_mode,
                                    ap if abc is not None else None, _ptrs(arrays)),
           "soaxref_fill_range")
    return arrays


def remove_flagged(schema, arrays, flags):
    """Sequential removal by overwriting with the last particle; returns the
    surviving prefix of every array (copies) and the new count."""
    arrays = [a.copy() for a in arrays]
    fl = np.ascontiguousarray(flags, dtype=np.uint8).copy()
    n = len(fl)
    m = lib().soaxref_remove_flagged(schema.ref, n, _ptrs(arrays) if arrays else None,
                                     fl.ctypes.data)
    if m < 0:
        raise ValueError("soaxref_remove_flagged failed")
    return [a[:m] for a in arrays], m


# Postfix op codes of the fused array expressions.
OP_ARRAY, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_NEG, OP_ABS, OP_SQRT, OP_MIN, OP_MAX = range(11)


def eval_program(arrays, prog, dst_dtype=np.float64):
    """A whole-array expression (the array access of Section 4.1, e.g.
    posArr(0) = velArr(1) - velArr(2)) applied element by element: the
    postfix program ``prog`` of (op, arg, value) triples is evaluated on a
    stack of float64 arrays in program order, one IEEE double operation per
    step (array elements converted to double first), and the result is
    rounded once to ``dst_dtype``.  MIN/MAX are (a < b ? a : b) and
    (a > b ? a : b)."""
    stack = []
    for op, arg, value in prog:
        if op == OP_ARRAY:
            stack.append(np.asarray(arrays[arg]).astype(np.float64))
        elif op == OP_CONST:
            n = len(arrays[0]) if arrays else 1
            stack.append(np.full(n, float(value), dtype=np.float64))
        elif op in (OP_NEG, OP_ABS, OP_SQRT):
            x = stack.pop()
            with np.errstate(invalid="ignore"):
                stack.append(-x if op == OP_NEG else np.abs(x) if op == OP_ABS else np.sqrt(x))
        else:
            b = stack.pop()
            a = stack.pop()
            with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
                if op == OP_ADD:
                    r = a + b
                elif op == OP_SUB:
                    r = a - b
                elif op == OP_MUL:
                    r = a * b
                elif op == OP_DIV:
                    r = a / b
                elif op == OP_MIN:
                    r = np.where(a < b, a, b)
                elif op == OP_MAX:
                    r = np.where(a > b, a, b)
                else:
                    raise ValueError(f"unknown op {op}")
            stack.append(r)
    if len(stack) != 1:
        raise ValueError("the program must leave exactly one value")
    with np.errstate(over="ignore"):
        return stack[0].astype(dst_dtype)


def field(abc, x):
    """u(x) for one point x (3,)."""
    a, ap = _abc(abc)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    u = np.zeros(3)
    lib().soaxref_field(ap, xx.ctypes.data, u.ctypes.data)
    return u


def step_soa(schema, arrays, integrator, dt, nsteps, abc=None, wrap=True):
    n = len(arrays[0]) if arrays else 0
    a, ap = _abc(abc)
    _check(lib().soaxref_step_soa(schema.ref, n, _ptrs(arrays), integrator, dt, nsteps, ap,
                                  int(wrap)), "soaxref_step_soa")


def step_aos(schema, aos, n, integrator, dt, nsteps, abc=None, wrap=True):
    assert aos.dtype == np.uint8 and aos.flags["C_CONTIGUOUS"]
    a, ap = _abc(abc)
    _check(lib().soaxref_step_aos(schema.ref, n, aos.ctypes.data, integrator, dt, nsteps, ap,
                                  int(wrap)), "soaxref_step_aos")


def aos_to_soa(schema, aos, n):
    arrays = empty_soa(schema, n)
    _check(lib().soaxref_aos_to_soa(schema.ref, n, aos.ctypes.data, _ptrs(arrays)),
           "soaxref_aos_to_soa")
    return arrays


def soa_to_aos(schema, arrays):
    n = len(arrays[0]) if arrays else 0
    _, stride = schema.layout()
    aos = np.full(n * stride, 0xA5, dtype=np.uint8)  # poison: every byte must be written
    _check(lib().soaxref_soa_to_aos(schema.ref, n, _ptrs(arrays), aos.ctypes.data),
           "soaxref_soa_to_aos")
    return aos


AOSOA_W = 64


def aosoa_layout(schema):
    """(byte offset of every SoA array inside a tile, tile bytes)."""
    narr = sum(d for _, _, d in schema.fields)
    off = (ctypes.c_int64 * max(narr, 1))()
    tile = ctypes.c_int64()
    _check(lib().soaxref_aosoa_layout(schema.ref, off, ctypes.byref(tile)), "soaxref_aosoa_layout")
    return list(off)[:narr], tile.value


def soa_to_aosoa(schema, arrays):
    n = len(arrays[0]) if arrays else 0
    _, tile = aosoa_layout(schema)
    out = np.full(-(-n // AOSOA_W) * tile, 0xA5, dtype=np.uint8)
    _check(lib().soaxref_soa_to_aosoa(schema.ref, n, _ptrs(arrays), out.ctypes.data),
           "soaxref_soa_to_aosoa")
    return out


def aosoa_to_soa(schema, buf, n):
    arrays = empty_soa(schema, n)
    _check(lib().soaxref_aosoa_to_soa(schema.ref, n, buf.ctypes.data, _ptrs(arrays)),
           "soaxref_aosoa_to_soa")
    return arrays


def rk2_forward(x0, abc, dt, nsteps, store_states=False):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = x0.shape[1]
    xT = np.zeros_like(x0)
    states = np.zeros((nsteps + 1, 3, n)) if store_states else None
    a, ap = _abc(abc)
    _check(lib().soaxref_rk2_forward(n, _rows(x0), _rows(xT), ap, dt, nsteps,
                                     states.ctypes.data if states is not None else None),
           "soaxref_rk2_forward")
    return (xT, states) if store_states else xT


def sqdist_loss(xT, target):
    xT = np.ascontiguousarray(xT, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    lam = np.zeros_like(xT)
    loss = lib().soaxref_sqdist_loss(xT.shape[1], _rows(xT), _rows(target), _rows(lam))
    return loss, lam


def _grad(fn, x0, lamT, abc, dt, nsteps):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    lamT = np.ascontiguousarray(lamT, dtype=np.float64)
    gx = np.zeros_like(x0)
    gabc = np.zeros(3)
    a, ap = _abc(abc)
    _check(fn(x0.shape[1], _rows(x0), _rows(lamT), ap, dt, nsteps, _rows(gx), gabc.ctypes.data),
           fn.__name__)
    return gx, gabc


def adjoint(x0, lamT, abc, dt, nsteps):
    """Reverse-mode gradients (store every state, one reverse sweep)."""
    return _grad(lib().soaxref_adjoint, x0, lamT, abc, dt, nsteps)


def tangent(x0, lamT, abc, dt, nsteps):
    """Forward-mode gradients (3x3 Jacobians carried along the trajectory)."""
    return _grad(lib().soaxref_tangent, x0, lamT, abc, dt, nsteps)


def mix64(z):
    return lib().soaxref_mix64(z)


def draw(seed, stream, i):
    return lib().soaxref_draw(seed, stream, i)
