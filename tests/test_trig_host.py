"""The library's fp64 sincos (csrc/trig.h) against glibc on the host: the
GPU kernels evaluate the same IEEE operations, so this bounds their error.
No GPU is used; the check program is compiled for the host with hipcc."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1710_03462_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("gcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("trig") / "trig_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-ffp-contract=off",
                    "-I", CSRC, os.path.join(HERE, "trig_check.cpp"), "-o", out],
                   check=True, capture_output=True)
    return out


@pytest.mark.parametrize("lo,hi", [(-1.0, 8.0), (-20.0, 20.0), (1e3, 1e4), (4e5, 5.2e5),
                                   (1e6, 1e9), (-1e-3, 1e-3)])
def test_sincos_within_two_ulp_of_glibc(exe, lo, hi):
    out = subprocess.run([exe, str(lo), str(hi), "400000"], check=True, capture_output=True,
                         text=True).stdout.split()
    worst_s, worst_c, shift_s, shift_c = float(out[0]), float(out[2]), float(out[4]), float(out[5])
    assert worst_s <= 2.0, out
    assert worst_c <= 2.0, out
    if hi - lo < 1e3:  # the shifted form: absolute error in units of ulp(1)
        assert shift_s <= 1.0 and shift_c <= 1.0, out
