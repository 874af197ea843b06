"""ctypes declarations of the C ABI in include/soax.h.

Loading fails loudly when libsoax.so has not been built: there is no
fallback implementation of any operation.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoax.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "soax.h")

SOAX_OK = 0
STATUS = {-1: "SOAX_E_ARG", -2: "SOAX_E_SCHEMA", -3: "SOAX_E_RANGE", -4: "SOAX_E_LAYOUT",
          -5: "SOAX_E_OOM", -6: "SOAX_E_HIP", -7: "SOAX_E_STATE"}
DTYPE = {"i8": 1, "u8": 2, "i32": 3, "i64": 4, "f32": 5, "f64": 6}
SOA, AOS, AOS_NAIVE, AOSOA = 0, 1, 2, 3
LAYOUTS = {"soa": SOA, "aos": AOS, "aos_naive": AOS_NAIVE, "aosoa": AOSOA}
EULER, EULER_ACC, RK2_ABC, HEUN_ABC, RK4_ABC, SYMPLECTIC_EULER = 0, 1, 2, 3, 4, 5
INTEGRATORS = {"euler": EULER, "euler_acc": EULER_ACC, "rk2_abc": RK2_ABC, "heun_abc": HEUN_ABC,
               "rk4_abc": RK4_ABC, "symplectic_euler": SYMPLECTIC_EULER}


class SoaxError(RuntimeError):
    def __init__(self, status, what, detail):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({detail})")


class Field(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("dtype", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("tag", ctypes.c_char)]


class SchemaC(ctypes.Structure):
    _fields_ = [("fields", ctypes.POINTER(Field)), ("nfields", ctypes.c_int32),
                ("packed", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("A", ctypes.c_double), ("B", ctypes.c_double), ("C", ctypes.c_double),
                ("wrap", ctypes.c_int32)]


_lib = None


def exported_names():
    """Function names declared in include/soax.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(soax_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1710_03462_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_double)
    sp = ctypes.POINTER(SchemaC)
    pp = ctypes.POINTER(Params)
    sigs = {
        "soax_schema_layout": [sp, vp, vp, vp],
        "soax_create": [sp, i64, vp],
        "soax_bind": [sp, i64, vp, vp, vp],
        "soax_destroy": [vp],
        "soax_layout_info": [vp, vp, vp, vp],
        "soax_buffer": [vp, i32, vp],
        "soax_fill": [vp, u64, i32, pp, vp],
        "soax_step": [vp, i32, i32, dbl, i64, pp, vp],
        "soax_step_fused": [vp, i32, dbl, i64, pp, vp],
        "soax_step_config": [vp, i32, i32, i32],
        "soax_aos_to_soa": [vp, vp],
        "soax_soa_to_aos": [vp, vp],
        "soax_get_record": [vp, i32, i64, vp],
        "soax_rk2_forward_ckpt": [vp, vp, i64, vp, dbl, i64, i64, vp, vp],
        "soax_adjoint": [vp, vp, i64, vp, dbl, i64, i64, vp, vp, vp],
        "soax_adjoint_noalloc": [vp, vp, i64, vp, dbl, i64, i64, vp, vp, vp],
        "soax_sqdist_loss": [vp, vp, i64, vp, vp, vp],
        "soax_batch_create": [vp, i32, vp],
        "soax_batch_destroy": [vp],
        "soax_batch_step": [vp, vp, vp, i64, i32, vp],
        "soax_batch_config": [vp, i32, i32, i32],
        "soax_batch_get_config": [vp, vp, vp, vp],
        "soax_batch_tune": [vp, ctypes.c_char_p],
        "soax_bind_capacity": [sp, i64, i64, vp, vp, vp],
        "soax_capacity": [vp, vp, vp],
        "soax_reserve": [vp, i64, vp],
        "soax_resize": [vp, i64, vp],
        "soax_push_back": [vp, vp, i64, vp],
        "soax_rebind": [vp, i64, vp, vp, vp],
        "soax_set_record": [vp, i64, vp],
        "soax_remove_flagged": [vp, vp, vp, vp],
        "soax_eval": [vp, i32, vp, i32, vp],
        "soax_eval_ptrs": [i64, vp, i32, vp, vp, i32, vp, i32, vp],
        "soax_expr_source": [vp, i32, i32, vp, i32, vp, i64],
        "soax_rk2_forward_ckpt_strided": [vp, vp, i64, i64, vp, dbl, i64, i64, vp, vp],
        "soax_adjoint_strided": [vp, vp, i64, i64, vp, dbl, i64, i64, vp, vp, vp],
        "soax_sqdist_loss_strided": [vp, i64, vp, i64, vp, vp, vp],
        "soax_aosoa_layout": [sp, vp, vp],
        "soax_bind_aosoa": [vp, vp, i64],
        "soax_soa_to_aosoa": [vp, vp],
        "soax_aosoa_to_soa": [vp, vp],
        "soax_step_graph_create": [vp, i32, i32, dbl, i64, pp, vp],
        "soax_step_graph_launch": [vp, vp],
        "soax_step_graph_destroy": [vp],
        "soax_copy": [vp, vp, i64, vp],
        "soax_probe": [i32, vp, vp, i64, vp],
        "soax_strerror": [i32],
        "soax_last_error": [],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    L.soax_destroy.restype = None
    L.soax_batch_destroy.restype = None
    L.soax_step_graph_destroy.restype = None
    L.soax_strerror.restype = ctypes.c_char_p
    L.soax_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status, what):
    if status != SOAX_OK:
        detail = lib().soax_last_error().decode(errors="replace")
        raise SoaxError(status, what, detail)
    return status


def make_schema(fields, packed=False):
    """(ctypes schema, keep-alive objects) for a list of (name, dtype, dim[, tag])."""
    arr = (Field * len(fields))()
    names = []
    for i, f in enumerate(fields):
        name, t, d = f[0], f[1], int(f[2])
        tag = f[3] if len(f) > 3 else name[:1]
        b = name.encode()
        names.append(b)
        code = t if isinstance(t, int) else DTYPE[t]
        arr[i] = Field(b, code, d, tag.encode()[:1] or b" ")
    sch = SchemaC(arr, len(fields), int(bool(packed)))
    return sch, (arr, names)
