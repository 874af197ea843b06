"""C-ABI checks that need no GPU: the library loads and exports every
function include/soax.h declares, its host-side record layout agrees with the
oracle's, and invalid calls return their documented status before any
device call is made."""
import ctypes
import math
import os

import pytest

import synth_inputs as si

soax = pytest.importorskip("paper_1710_03462_amd")
from paper_1710_03462_amd import _lib  # noqa: E402

E_ARG, E_SCHEMA, E_RANGE, E_LAYOUT = -1, -2, -3, -4
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L(host_lib):
    return host_lib


def test_exports_every_declared_function(L):
    names = _lib.exported_names()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name


def test_header_declarations_match_binding_signatures():
    declared = set(_lib.exported_names())
    bound = {"soax_schema_layout", "soax_create", "soax_bind", "soax_destroy", "soax_layout_info",
             "soax_buffer", "soax_fill", "soax_step", "soax_step_config", "soax_aos_to_soa",
             "soax_soa_to_aos", "soax_get_record", "soax_rk2_forward_ckpt", "soax_adjoint",
             "soax_sqdist_loss", "soax_batch_create", "soax_batch_destroy", "soax_batch_step",
             "soax_batch_config", "soax_batch_get_config", "soax_batch_tune", "soax_copy",
             "soax_strerror", "soax_last_error", "soax_bind_capacity", "soax_capacity",
             "soax_reserve", "soax_resize", "soax_push_back", "soax_rebind", "soax_set_record",
             "soax_remove_flagged", "soax_eval", "soax_eval_ptrs", "soax_expr_source",
             "soax_rk2_forward_ckpt_strided", "soax_adjoint_strided", "soax_sqdist_loss_strided",
             "soax_aosoa_layout", "soax_bind_aosoa", "soax_soa_to_aosoa", "soax_aosoa_to_soa",
             "soax_step_graph_create", "soax_step_graph_launch", "soax_step_graph_destroy",
             "soax_adjoint_noalloc", "soax_probe", "soax_step_fused"}
    assert declared == bound


SCHEMAS = [si.BASE_FIELDS, si.WIDE_FIELDS, si.particle_size_fields(5),
           [("a", "u8", 1), ("b", "i64", 1), ("c", "i8", 3), ("d", "f32", 2)]]


@pytest.mark.parametrize("k", range(len(SCHEMAS)))
@pytest.mark.parametrize("packed", [False, True])
def test_layout_agrees_with_oracle(ref, k, packed):
    fields = SCHEMAS[k]
    off, stride, soa_bytes = soax.Schema(fields, packed).layout()
    roff, rstride = ref.Schema(fields, packed).layout()
    assert (off, stride) == (roff, rstride)
    assert soa_bytes == sum({"i8": 1, "u8": 1, "i32": 4, "i64": 8, "f32": 4, "f64": 8}[t] * d
                            for _, t, d in fields)


def _status(fn, *args):
    return fn(*args)


def test_schema_errors(L):
    def code(fields, packed=False):
        sch, keep = _lib.make_schema(fields, packed)
        return L.soax_schema_layout(ctypes.byref(sch), None, None, None)

    assert code([("x", "f64", 3)]) == 0
    assert code([("x", "f64", 4)]) == E_SCHEMA
    assert code([("x", "f64", 0)]) == E_SCHEMA
    assert code([("x", 9, 1)]) == E_SCHEMA
    assert code([("x", "f64", 1), ("x", "f32", 1)]) == E_SCHEMA
    assert code([("", "f64", 1)]) == E_SCHEMA
    assert code([("n" * 40, "f64", 1)]) == E_SCHEMA
    assert code([(f"f{i}", "f32", 1) for i in range(33)]) == E_SCHEMA
    assert L.soax_schema_layout(None, None, None, None) == E_ARG
    assert b"schema" in L.soax_last_error()


def test_create_and_bind_argument_errors(L):
    sch, keep = _lib.make_schema(si.BASE_FIELDS)
    h = ctypes.c_void_p()
    assert L.soax_create(ctypes.byref(sch), -1, ctypes.byref(h)) == E_ARG
    assert L.soax_create(ctypes.byref(sch), 2 ** 31, ctypes.byref(h)) == E_RANGE
    assert L.soax_create(ctypes.byref(sch), 10, None) == E_ARG
    assert L.soax_bind(ctypes.byref(sch), 10, None, None, ctypes.byref(h)) == E_ARG
    ptrs = (ctypes.c_void_p * 7)(*([0x10000] * 6 + [0]))
    assert L.soax_bind(ctypes.byref(sch), 10, ptrs, None, ctypes.byref(h)) == E_ARG
    sch8, keep8 = _lib.make_schema([("id", "u8", 1), ("pos", "f64", 3), ("vel", "f32", 3)])
    assert L.soax_create(ctypes.byref(sch8), 1000, ctypes.byref(h)) == E_RANGE


@pytest.fixture
def soa_only_set(L):
    """A set bound to placeholder SoA addresses and no AoS copy: binding it
    makes no device call, and every call below must fail validation before
    touching those addresses."""
    made = []

    def make(fields):
        sch, keep = _lib.make_schema(fields)
        narr = sum(int(f[2]) for f in fields)
        ptrs = (ctypes.c_void_p * narr)(*[0x100000 * (a + 1) for a in range(narr)])
        h = ctypes.c_void_p()
        assert L.soax_bind(ctypes.byref(sch), 1000, ptrs, None, ctypes.byref(h)) == 0
        made.append((h, sch, keep))
        return h

    yield make
    for h, _, _ in made:
        L.soax_destroy(h)


def test_step_validation(L, soa_only_set):
    h = soa_only_set(si.BASE_FIELDS)
    p = _lib.Params(1.0, 1.0, 1.0, 1)
    bad = _lib.Params(math.nan, 1.0, 1.0, 1)
    s = ctypes.byref
    assert L.soax_step(h, 4, 0, 1e-3, 1, s(p), None) == E_ARG          # unknown layout
    assert L.soax_step(h, 3, 0, 1e-3, 1, s(p), None) == E_LAYOUT       # no AoSoA copy bound
    assert L.soax_soa_to_aosoa(h, None) == E_LAYOUT
    assert L.soax_bind_aosoa(h, ctypes.c_void_p(0x400000), 100) == E_ARG  # too small
    assert L.soax_bind_aosoa(h, ctypes.c_void_p(0x400008), 1 << 20) == E_LAYOUT  # misaligned
    assert L.soax_step(h, 0, 7, 1e-3, 1, s(p), None) == E_ARG          # unknown integrator
    assert L.soax_step(h, 0, 0, math.inf, 1, s(p), None) == E_ARG      # dt
    assert L.soax_step(h, 0, 0, 1e-3, -1, s(p), None) == E_ARG         # nsteps
    assert L.soax_step(h, 0, 2, 1e-3, 1, None, None) == E_ARG          # RK2 needs params
    assert L.soax_step(h, 0, 2, 1e-3, 1, s(bad), None) == E_ARG        # amplitudes
    assert L.soax_step(h, 0, 1, 1e-3, 1, s(p), None) == E_SCHEMA       # no acc
    assert L.soax_step(h, 1, 0, 1e-3, 1, s(p), None) == E_LAYOUT       # no AoS copy
    assert L.soax_step(h, 2, 0, 1e-3, 1, s(p), None) == E_LAYOUT
    assert L.soax_aos_to_soa(h, None) == E_LAYOUT
    assert L.soax_soa_to_aos(h, None) == E_LAYOUT
    assert L.soax_fill(h, 0, 2, None, None) == E_ARG
    assert L.soax_step_config(h, 0, 100, 0) == E_ARG
    assert L.soax_step_config(h, 0, 256, 3) == E_ARG
    assert L.soax_step_config(h, 1, 256, 2) == E_ARG
    assert L.soax_step_config(h, 0, 256, 2) == 0
    rec = (ctypes.c_uint8 * 48)()
    assert L.soax_get_record(h, 0, 1000, rec) == E_ARG
    assert L.soax_get_record(h, 1, 0, rec) == E_LAYOUT
    assert b"AoS" in L.soax_last_error()


def test_step_type_rules(L, soa_only_set):
    p = _lib.Params(1.0, 1.0, 1.0, 1)
    f32pos = soa_only_set(si.particle_size_fields(0))
    assert L.soax_step(f32pos, 0, 2, 1e-3, 1, ctypes.byref(p), None) == E_SCHEMA  # RK2 needs f64
    assert L.soax_step(f32pos, 0, 0, 1e-3, 1, ctypes.byref(p), None) == E_SCHEMA  # wrap needs f64
    mixed = soa_only_set([("pos", "f64", 3), ("vel", "f32", 3), ("acc", "f64", 3)])
    assert L.soax_step(mixed, 0, 1, 1e-3, 1, ctypes.byref(p), None) == E_SCHEMA
    novel = soa_only_set([("pos", "f64", 3)])
    assert L.soax_step(novel, 0, 0, 1e-3, 1, None, None) == E_SCHEMA


def test_adjoint_and_loss_validation(L):
    rows = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    none3 = (ctypes.c_void_p * 3)(0x1000, None, 0x3000)
    abc = (ctypes.c_double * 3)(1.0, 0.8, 0.6)
    nan = (ctypes.c_double * 3)(1.0, math.nan, 0.6)
    tape = ctypes.c_void_p(0x4000)
    f = L.soax_rk2_forward_ckpt
    assert f(rows, rows, 10, abc, 5e-3, 20, 0, tape, None) == E_ARG       # k < 1
    assert f(rows, rows, 10, abc, 5e-3, -1, 5, tape, None) == E_ARG
    assert f(rows, rows, 10, nan, 5e-3, 20, 5, tape, None) == E_ARG
    assert f(none3, rows, 10, abc, 5e-3, 20, 5, tape, None) == E_ARG
    assert f(rows, rows, 10, abc, 5e-3, 20, 5, None, None) == E_ARG
    assert f(rows, rows, -1, abc, 5e-3, 20, 5, tape, None) == E_ARG
    assert f(rows, rows, 2 ** 31, abc, 5e-3, 20, 5, tape, None) == E_RANGE
    a = L.soax_adjoint
    assert a(tape, rows, 10, abc, 5e-3, 20, 5, rows, None, None) == E_ARG  # grad_abc
    assert a(tape, rows, 10, abc, math.nan, 20, 5, rows, tape, None) == E_ARG
    assert a(tape, none3, 10, abc, 5e-3, 20, 5, rows, tape, None) == E_ARG
    assert L.soax_sqdist_loss(rows, rows, 10, None, None, None) == E_ARG
    # the allocation-free adjoint: its argument checks and its size limit are
    # decided on the host, before any device call
    z = L.soax_adjoint_noalloc
    assert z(tape, rows, 10, abc, 5e-3, 20, 5, rows, None, None) == E_ARG
    assert z(tape, rows, 10, abc, 5e-3, 20, 0, rows, tape, None) == E_ARG
    assert z(tape, rows, -1, abc, 5e-3, 20, 5, rows, tape, None) == E_ARG
    assert z(tape, rows, 11184640 + 1, abc, 5e-3, 20, 5, rows, tape, None) == E_RANGE
    assert b"scratch" in L.soax_last_error()


def test_copy_and_batch_validation(L):
    assert L.soax_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 64, None) == E_ARG
    assert L.soax_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), -1, None) == E_ARG
    assert L.soax_copy(None, None, 0, None) == 0
    rows = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    none3 = (ctypes.c_void_p * 3)(0x1000, None, 0x3000)
    assert L.soax_probe(4, rows, rows, 10, None) == E_ARG
    assert L.soax_probe(0, rows, none3, 10, None) == E_ARG
    assert L.soax_probe(0, none3, rows, 10, None) == E_ARG
    assert L.soax_probe(1, rows, rows, -1, None) == E_ARG
    assert L.soax_probe(0, rows, rows, 2 ** 31, None) == E_RANGE
    assert L.soax_probe(2, None, None, 0, None) == 0
    h = ctypes.c_void_p()
    assert L.soax_batch_create(None, 0, ctypes.byref(h)) == E_ARG
    arr = (ctypes.c_void_p * 1)(None)
    assert L.soax_batch_create(arr, 1, ctypes.byref(h)) == E_ARG
    assert L.soax_batch_step(None, None, None, 1, 2, None) == E_ARG


def test_strerror(L):
    assert L.soax_strerror(0) == b"ok"
    assert L.soax_strerror(-4) == b"layout unavailable"
    assert L.soax_strerror(-99) == b"unknown status"


E_STATE = -7


def test_container_validation(L, soa_only_set):
    """Container calls on a bound set reject what they cannot do before any
    device call: growing past the bound capacity, bad sizes, null buffers."""
    h = soa_only_set(si.BASE_FIELDS)  # 1000 particles, capacity 1000, no AoS copy
    n, cap = ctypes.c_int64(), ctypes.c_int64()
    assert L.soax_capacity(h, ctypes.byref(n), ctypes.byref(cap)) == 0
    assert (n.value, cap.value) == (1000, 1000)
    assert L.soax_capacity(None, None, None) == E_ARG
    assert L.soax_resize(h, -1, None) == E_ARG
    assert L.soax_resize(h, 2 ** 31, None) == E_RANGE
    assert L.soax_resize(h, 1001, None) == E_STATE        # bound sets do not grow
    assert b"bound" in L.soax_last_error()
    assert L.soax_reserve(h, 5000, None) == E_STATE
    assert L.soax_reserve(h, 10, None) == 0               # never shrinks: no-op
    rec = (ctypes.c_uint8 * 48)()
    assert L.soax_push_back(h, rec, -1, None) == E_ARG
    assert L.soax_push_back(h, None, 1, None) == E_ARG
    assert L.soax_push_back(h, rec, 1, None) == E_STATE
    assert L.soax_set_record(h, 1000, rec) == E_ARG
    new_n = ctypes.c_int64()
    assert L.soax_remove_flagged(h, None, ctypes.byref(new_n), None) == E_ARG
    assert L.soax_remove_flagged(h, None, None, None) == E_ARG
    assert L.soax_rebind(h, 999, None, None, None) == E_ARG    # below n
    assert L.soax_rebind(h, 2000, None, None, None) == E_LAYOUT  # the SoA copy is missing
    ptrs = (ctypes.c_void_p * 7)(*[0x200000 * (a + 1) for a in range(7)])
    assert L.soax_rebind(h, 2000, ptrs, ctypes.c_void_p(0x9000000), None) == E_LAYOUT  # AoS added
    assert L.soax_capacity(h, ctypes.byref(n), ctypes.byref(cap)) == 0
    assert (n.value, cap.value) == (1000, 1000)            # nothing changed


def test_bind_capacity_validation(L):
    sch, keep = _lib.make_schema(si.BASE_FIELDS)
    ptrs = (ctypes.c_void_p * 7)(*[0x100000 * (a + 1) for a in range(7)])
    h = ctypes.c_void_p()
    assert L.soax_bind_capacity(ctypes.byref(sch), 10, 5, ptrs, None, ctypes.byref(h)) == E_ARG
    assert L.soax_bind_capacity(ctypes.byref(sch), 10, 2 ** 31, ptrs, None, ctypes.byref(h)) == E_RANGE
    assert L.soax_bind_capacity(ctypes.byref(sch), 10, 64, ptrs, None, ctypes.byref(h)) == 0
    n, cap = ctypes.c_int64(), ctypes.c_int64()
    assert L.soax_capacity(h, ctypes.byref(n), ctypes.byref(cap)) == 0
    assert (n.value, cap.value) == (10, 64)
    L.soax_destroy(h)


def test_aosoa_layout_agrees_with_oracle(ref, L):
    for fields in SCHEMAS:
        sch, keep = _lib.make_schema(fields)
        narr = sum(int(f[2]) for f in fields)
        off = (ctypes.c_int64 * narr)()
        tile = ctypes.c_int64()
        assert L.soax_aosoa_layout(ctypes.byref(sch), off, ctypes.byref(tile)) == 0
        roff, rtile = ref.aosoa_layout(ref.Schema(fields))
        assert (list(off), tile.value) == (roff, rtile)


def test_product_fails_loudly_without_the_library(tmp_path):
    """With libsoax.so absent the package raises on first use: there is no
    fallback implementation anywhere."""
    import subprocess
    import sys
    code = ("import paper_1710_03462_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/libsoax.so'\n"
            "L._lib = None\n"
            "try:\n"
            "    L.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', 'no CPU fallback' in str(e))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=str(tmp_path), env={"PYTHONPATH": ROOT, "PATH": "/usr/bin:/bin"})
    assert "raised: True" in r.stdout, r.stdout + r.stderr


def test_product_never_imports_the_oracle(host_lib):
    import subprocess
    import sys
    code = ("import sys, paper_1710_03462_amd as s\n"
            "s.lib(); s.Schema([('id', 'i32', 1), ('pos', 'f64', 3), ('vel', 'f32', 3)]).layout()\n"
            "import bench\n"
            "print('oracle' in sys.modules)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       env={"PYTHONPATH": ROOT, "PATH": "/usr/bin:/bin"})
    assert r.stdout.strip().endswith("False"), r.stdout + r.stderr
