"""Build the device-side check helpers the GPU tests load (test
infrastructure, not part of the library): trig_device_check.hip ->
tests/libtrig_device_check.so, compiled for gfx950 with the library's own
floating-point flags so that the device code under test is built the same
way as in libsoax.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1710_03462_amd", "csrc")
TRIG_SRC = os.path.join(HERE, "trig_device_check.hip")
TRIG_LIB = os.path.join(HERE, "libtrig_device_check.so")


def build(verbose=False):
    sys.path.insert(0, ROOT)
    from paper_1710_03462_amd.build import FLAGS, HIPCC
    tmp = TRIG_LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", TRIG_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on trig_device_check.hip:\n" + r.stderr)
    os.replace(tmp, TRIG_LIB)
    return TRIG_LIB


if __name__ == "__main__":
    build(verbose=True)
