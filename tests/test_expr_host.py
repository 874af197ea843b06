"""Host-side checks of the fused array expressions: invalid programs are
rejected before any device call, and the kernel source the library
generates for every op and element type compiles for gfx950 (with the same
compiler the library's run-time compilation uses).  No GPU is used."""
import ctypes
import os

import pytest

soax = pytest.importorskip("paper_1710_03462_amd")
from paper_1710_03462_amd import _lib  # noqa: E402
from paper_1710_03462_amd import expr as E  # noqa: E402

E_ARG, E_SCHEMA = -1, -2


@pytest.fixture(autouse=True)
def _built(host_lib):
    """Every test here calls the library through _lib.lib()."""


def prog(*ops):
    arr = (E.ExprOp * len(ops))()
    for i, o in enumerate(ops):
        arr[i] = E.ExprOp(*o)
    return arr


def src_status(p, nops=None, dst=6, types=(6,), size=1 << 16):
    L = _lib.lib()
    t = (ctypes.c_int32 * max(len(types), 1))(*types)
    buf = ctypes.create_string_buffer(size)
    return L.soax_expr_source(p, len(p) if nops is None else nops, dst, t, len(types), buf, size)


def test_program_validation():
    ok = prog((E.ARRAY, 0, 0), (E.CONST, 0, 2.0), (E.MUL, 0, 0))
    assert src_status(ok) == 0
    assert src_status(prog((E.ARRAY, 1, 0))) == E_ARG                  # array out of range
    assert src_status(prog((E.ARRAY, 0, 0), (E.ADD, 0, 0))) == E_ARG   # underflow
    assert src_status(prog((E.ARRAY, 0, 0), (E.ARRAY, 0, 0))) == E_ARG  # two values left
    assert src_status(prog((E.ARRAY, 0, 0), (99, 0, 0))) == E_ARG      # unknown op
    assert src_status(ok, nops=0) == E_ARG
    assert src_status(ok, dst=3) == E_SCHEMA                          # integer destination
    assert src_status(ok, types=(9,)) == E_SCHEMA                     # unknown source type
    assert src_status(ok, size=16) == E_ARG                           # buffer too small
    many = prog(*([(E.CONST, 0, 1.0)] + [(E.CONST, 0, 1.0), (E.ADD, 0, 0)] * 32))
    assert src_status(many, types=()) == E_ARG                        # 33 constants
    L = _lib.lib()
    assert L.soax_eval_ptrs(-1, None, 6, None, None, 0, ok, 3, None) == E_ARG
    assert L.soax_eval_ptrs(10, None, 6, None, None, 0, ok, 3, None) == E_ARG  # null dst
    assert L.soax_eval(None, 0, ok, 3, None) == E_ARG


def hiprtc_compile(src):
    """Compile with hipRTC exactly as the library does; returns (ok, log)."""
    path = "/opt/rocm/lib/libhiprtc.so"
    if not os.path.exists(path):
        pytest.skip("hipRTC not available")
    rtc = ctypes.CDLL(path)
    prog = ctypes.c_void_p()
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"gen.hip", 0, None, None) == 0
    opts = [b"--offload-arch=gfx950", b"-O3", b"-ffp-contract=off", b"-Xclang", b"-target-feature",
            b"-Xclang", b"-packed-fp32-ops"]
    arr = (ctypes.c_char_p * len(opts))(*opts)
    rc = rtc.hiprtcCompileProgram(prog, len(opts), arr)
    n = ctypes.c_size_t()
    rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(n))
    log = ctypes.create_string_buffer(max(n.value, 1))
    rtc.hiprtcGetProgramLog(prog, log)
    size = ctypes.c_size_t()
    rtc.hiprtcGetCodeSize(prog, ctypes.byref(size))
    rtc.hiprtcDestroyProgram(ctypes.byref(prog))
    return rc == 0 and size.value > 0, log.value.decode(errors="replace")


@pytest.mark.parametrize("dst", ["f32", "f64"])
def test_generated_source_compiles_for_gfx950(dst):
    a, b, c, d, e, f = (E.array(k) for k in "abcdef")
    ex = E.sqrt(abs(a * b + 1.5 / c)) - E.minimum(d, E.maximum(e, -f)) + (2.0 - a)
    src = E.source(ex, dst, ["i8", "u8", "i32", "i64", "f32", "f64"])
    for t in ("signed char", "unsigned char", "int", "long long", "float", "double"):
        assert f"(const {t}*)" in src
    ok, log = hiprtc_compile(src)
    assert ok, log


def test_builder_operand_order():
    a, b = E.array("a"), E.array("b")
    steps = [op for op, _, _ in (3.0 - a / b).steps]
    assert steps == [E.CONST, E.ARRAY, E.ARRAY, E.DIV, E.SUB]
    assert (a - 1.0).steps[-2][0] == E.CONST and (a - 1.0).steps[0][0] == E.ARRAY
    assert (a * a).keys() == ["a"]
