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
