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
                                   (-5.2e5, -4e5), (1e6, 1e9), (-1e9, -1e6), (-1e-3, 1e-3)])
def test_sincos_within_two_ulp_of_glibc(exe, lo, hi):
    out = subprocess.run([exe, str(lo), str(hi), "400000"], check=True, capture_output=True,
                         text=True).stdout.split()
    worst_s, worst_c, shift_s, shift_c = float(out[0]), float(out[2]), float(out[4]), float(out[5])
    assert worst_s <= 2.0, out
    assert worst_c <= 2.0, out
    if hi - lo < 1e3:  # the shifted form: absolute error in units of ulp(1)
        assert shift_s <= 1.0 and shift_c <= 1.0, out


@pytest.mark.parametrize("lo,hi", [(-1.0, 8.0), (-20.0, 20.0), (-1e-3, 1e-3)])
def test_checked_shift_longer_series_within_one_ulp(exe, lo, hi):
    # shifts up to 1/8: the degree-9/10 series of the mid and unbounded tiers
    # keeps the absolute error of sin/cos(x + d) within one ulp of 1
    out = subprocess.run([exe, str(lo), str(hi), "400000", str(1.0 / 8)], check=True,
                         capture_output=True, text=True).stdout.split()
    assert float(out[4]) <= 1.0 and float(out[5]) <= 1.0, out


@pytest.mark.parametrize("shift_max", [1.0 / 64, 1.0 / 8, 0.5])
def test_mid_tier_equals_the_any_tier_inside_its_bound(exe, shift_max):
    # kTierMid (|d| <= 1/8) drops the range check the host has proven
    # unneeded; inside that bound it must give the any-tier results bit for
    # bit (field 6: count of differing pairs)
    out = subprocess.run([exe, "-20", "20", "400000", str(shift_max)], check=True,
                         capture_output=True, text=True).stdout.split()
    assert int(out[6]) == 0, out


@pytest.mark.parametrize("lo,hi", [(-1.0, 8.0), (-20.0, 20.0), (-1e-3, 1e-3)])
def test_small_tier_short_series_within_one_ulp(exe, lo, hi):
    # kTierSmall's degree-5/6 series for |d| <= 1/64 (field 7: its largest
    # absolute error in units of ulp(1) against long double)
    out = subprocess.run([exe, str(lo), str(hi), "400000", str(1.0 / 64)], check=True,
                         capture_output=True, text=True).stdout.split()
    assert float(out[7]) <= 1.0, out


@pytest.mark.parametrize("lo,hi", [(-1.0, 8.0), (-20.0, 20.0)])
def test_checked_shift_full_reduction_beyond_the_series(exe, lo, hi):
    # shifts up to 1/2 reach the full reduction of the rounded sum x + d: its
    # error is at most half an ulp of x + d (the rounding of the sum) plus the
    # reduction's own, in units of ulp(1)
    import math
    out = subprocess.run([exe, str(lo), str(hi), "400000", "0.5"], check=True,
                         capture_output=True, text=True).stdout.split()
    top = max(abs(lo), abs(hi)) + 0.5
    bound = 1.0 + 0.5 * math.ulp(top) / 2.0 ** -52 + 1.0
    assert float(out[4]) <= bound and float(out[5]) <= bound, (out, bound)


@pytest.mark.parametrize("dt,abc,tier", [
    (1e-3, (1, 1, 1), 0),                       # 3e-3: short series
    (1.0 / 192, (1, 1, 1), 0),                  # exactly 1/64
    (1.0 / 192 * (1 + 2.0 ** -40), (1, 1, 1), 1),
    (0.04, (1, 1, 1), 1),                       # 0.12
    (0.125 / 3 * (1 - 2.0 ** -19), (1, 1, 1), 1),
    (0.125 / 3 * (1 - 2.0 ** -22), (1, 1, 1), 2),  # inside 1/8 but within the 2^-20 margin
    (0.05, (1, 1, 1), 2),
    (-0.04, (-1, 1, -1), 1),                    # signs do not matter
    (1e-2, (0, 0, 0), 0),                       # no field
])
def test_shift_tier_selection(exe, dt, abc, tier):
    # the host's proof of the step's shift bound: |dt| (|A|+|B|+|C|) <= 1/64
    # -> 0, <= 1/8 (1 - 2^-20) -> 1, else 2
    out = subprocess.run([exe, "tier", repr(dt), *(repr(float(a)) for a in abc)], check=True,
                         capture_output=True, text=True).stdout.split()
    assert int(out[0]) == tier, (dt, abc, out)
