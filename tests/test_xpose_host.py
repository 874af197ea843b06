"""The transpose table's grouping of arrays by element size (launch.h),
compiled for the host: every array appears once, 8-byte arrays first, then
4-byte, then 1-byte, each group in schema order.  No GPU is used."""
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
    out = str(tmp_path_factory.mktemp("xpose") / "xpose_order_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I", CSRC,
                    os.path.join(HERE, "xpose_order_check.cpp"), "-o", out],
                   check=True, capture_output=True)
    return out


@pytest.mark.parametrize("sizes", [
    [4, 8, 8, 8, 4, 4, 4],              # base record: id, pos, vel
    [8, 4, 8, 8, 8, 4, 4, 4, 4, 4, 4, 8, 1],  # wide record
    [1, 8, 1, 1, 1, 4, 4],              # bytes-heavy schema
    [4] * 11,                           # Particle<5>
    [1],
])
def test_groups_by_size_in_schema_order(exe, sizes):
    out = subprocess.run([exe, *map(str, sizes)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    order = [int(v) for v in out[0].split()]
    ends = [int(v) for v in out[1].split()]
    want = [a for es in (8, 4, 1) for a, s in enumerate(sizes) if s == es]
    assert order == want
    assert ends == [sum(s == 8 for s in sizes), sum(s in (8, 4) for s in sizes), len(sizes)]
