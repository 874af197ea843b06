"""The GPU's sine/cosine (the inline-asm fma chain of csrc/trig.h) against the
host build of the same header, bit for bit.  Both evaluate the same chain of
correctly rounded fused multiply-adds, so any difference -- a swapped series
constant, a wrong operand in the asm block -- shows as a mismatch, even one
far below the 1e-12 tolerance of the particle parity tests.  The host branch
is itself bounded against glibc and long double by test_trig_host.py."""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtrig_device_check.so")
KINDS = ["sin x", "cos x", "sin(x+d) small tier", "cos(x+d) small tier", "sin(x+e) any tier",
         "cos(x+e) any tier", "sin(x+f) mid tier", "cos(x+f) mid tier"]

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def check():
    if not os.path.exists(LIB):
        pytest.fail("tests/libtrig_device_check.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    fn = lib.trig_device_check
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                   ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    return fn


# ranges of the fast path (|x| <= 2^19); shifts up to 1/8 take the longer
# series, any-tier shifts up to 1/2 also the full reduction of x + e
@pytest.mark.parametrize("lo,hi", [(-1.0, 8.0), (-20.0, 20.0), (1e3, 1e4), (4e5, 5.2e5),
                                   (-5.2e5, -4e5), (-1e-3, 1e-3)])
@pytest.mark.parametrize("emax", [1.0 / 64, 1.0 / 8, 0.5])
def test_device_sincos_bit_equal_to_host(check, lo, hi, emax):
    n = 1 << 18
    mism = np.zeros(len(KINDS), dtype=np.int64)
    first = np.zeros(len(KINDS), dtype=np.float64)
    print(f"trig_device_check n={n} range=({lo}, {hi}) emax={emax}", flush=True)
    rc = check(n, lo, hi, emax, 12345, mism.ctypes.data, first.ctypes.data)
    assert rc == 0, f"HIP error {rc}"
    bad = {KINDS[k]: (int(mism[k]), float(first[k])) for k in range(len(KINDS)) if mism[k]}
    assert not bad, bad
