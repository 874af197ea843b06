"""Shared test set-up: the ``gpu`` marker and import paths.

Tests marked ``gpu`` need an MI355X and the built HIP library; everything
else runs on the CPU (oracle pins, host-side layout logic, C-ABI symbol and
argument checks that return before any device call).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built HIP library")


@pytest.fixture(scope="session")
def ref():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def host_lib():
    """libsoax.so for the CPU-only C-ABI tests, compiled here first if this
    checkout has not been built (hipcc cross-compiles for gfx950 without a
    GPU).  GPU tests load the library that was built beforehand."""
    from paper_1710_03462_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.lib()
