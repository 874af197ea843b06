"""Fused element-wise array expressions (the whole-array expressions of
Section 4.1, evaluated in one kernel like the expression templates of
Section 4.2).

Arithmetic on `Expr` objects only records a postfix program; nothing is
computed until the program is handed to the library, which compiles one
kernel for it:

    ps = ParticleSet(fields, n)
    ps.assign(("pos", 0), ps.arr("vel", 1) - ps.arr("vel", 2))
    evaluate(out, sqrt(array(a) * array(a) + array(b) * array(b)))
"""
import ctypes

import torch

from . import _lib
from ._lib import check, lib

ARRAY, CONST, ADD, SUB, MUL, DIV, NEG, ABS, SQRT, MIN, MAX = range(11)
OP_NAMES = {ADD: "+", SUB: "-", MUL: "*", DIV: "/", NEG: "neg", ABS: "abs", SQRT: "sqrt",
            MIN: "min", MAX: "max"}

_DTYPE_CODE = {torch.int8: 1, torch.uint8: 2, torch.int32: 3, torch.int64: 4, torch.float32: 5,
               torch.float64: 6}


class ExprOp(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("arg", ctypes.c_int32), ("value", ctypes.c_double)]


class Expr:
    """A postfix program; ARRAY steps carry a key naming their array."""

    def __init__(self, steps):
        self.steps = list(steps)

    def _bin(self, other, op, reverse=False):
        o = as_expr(other)
        a, b = (o, self) if reverse else (self, o)
        return Expr(a.steps + b.steps + [(op, None, 0.0)])

    def __add__(self, o): return self._bin(o, ADD)
    def __radd__(self, o): return self._bin(o, ADD, True)
    def __sub__(self, o): return self._bin(o, SUB)
    def __rsub__(self, o): return self._bin(o, SUB, True)
    def __mul__(self, o): return self._bin(o, MUL)
    def __rmul__(self, o): return self._bin(o, MUL, True)
    def __truediv__(self, o): return self._bin(o, DIV)
    def __rtruediv__(self, o): return self._bin(o, DIV, True)
    def __neg__(self): return Expr(self.steps + [(NEG, None, 0.0)])
    def __abs__(self): return Expr(self.steps + [(ABS, None, 0.0)])

    def keys(self):
        """The distinct array keys in order of first use (tensors by identity,
        other keys by equality)."""
        out = []
        for op, key, _ in self.steps:
            if op == ARRAY and not any(_same(key, k) for k in out):
                out.append(key)
        return out

    def program(self, index_of):
        """ctypes array of ops, ARRAY args given by index_of(key)."""
        arr = (ExprOp * len(self.steps))()
        for i, (op, key, value) in enumerate(self.steps):
            arr[i] = ExprOp(op, index_of(key) if op == ARRAY else 0, float(value))
        return arr

    def as_tuples(self, index_of):
        return [(op, index_of(key) if op == ARRAY else 0, float(value))
                for op, key, value in self.steps]


def _same(a, b):
    if isinstance(a, torch.Tensor) or isinstance(b, torch.Tensor):
        return a is b
    return a == b


def as_expr(x):
    if isinstance(x, Expr):
        return x
    if isinstance(x, torch.Tensor):
        raise TypeError("wrap a tensor with array() to use it in an expression")
    return Expr([(CONST, None, float(x))])


def sqrt(e):
    return Expr(as_expr(e).steps + [(SQRT, None, 0.0)])


def minimum(a, b):
    return as_expr(a)._bin(b, MIN)


def maximum(a, b):
    return as_expr(a)._bin(b, MAX)


def array(t):
    """An array as an expression leaf: a device tensor for evaluate(), or any
    key for source()."""
    return Expr([(ARRAY, t, 0.0)])


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def evaluate(dst, expr):
    """dst[i] = expr(i) over plain contiguous device tensors of one length."""
    expr = as_expr(expr)
    keys = expr.keys()
    n = dst.numel()
    for t in keys:
        if not isinstance(t, torch.Tensor) or t.numel() != n or not t.is_contiguous():
            raise ValueError("every array must be a contiguous tensor of dst's length")
    if dst.dtype not in (torch.float32, torch.float64) or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous float32 or float64 tensor")

    def index_of(key):
        for j, k in enumerate(keys):
            if k is key:
                return j
        raise KeyError(key)

    prog = expr.program(index_of)
    src = (ctypes.c_void_p * max(len(keys), 1))(*[t.data_ptr() for t in keys])
    types = (ctypes.c_int32 * max(len(keys), 1))(*[_DTYPE_CODE[t.dtype] for t in keys])
    check(lib().soax_eval_ptrs(n, ctypes.c_void_p(dst.data_ptr()), _DTYPE_CODE[dst.dtype], src,
                               types, len(keys), prog, len(prog), _stream()), "soax_eval_ptrs")


def source(expr, dst_dtype="f64", src_dtypes=()):
    """The HIP source the library generates for a program (host only)."""
    expr = as_expr(expr)
    keys = expr.keys()
    prog = expr.program(lambda key: next(j for j, k in enumerate(keys) if _same(k, key)))
    types = (ctypes.c_int32 * max(len(src_dtypes), 1))(*[_lib.DTYPE[t] for t in src_dtypes])
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib().soax_expr_source(prog, len(prog), _lib.DTYPE[dst_dtype], types, len(src_dtypes),
                                 buf, len(buf)), "soax_expr_source")
    return buf.value.decode()
