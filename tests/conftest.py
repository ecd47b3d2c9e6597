import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionstart(session):
    """Build the HIP library once if it is missing (a fresh checkout); a library
    that is already built is used as it is."""
    lib = os.path.join(ROOT, "paper_1805_12498_amd", "libhafgpu.so")
    if not os.path.exists(lib):
        from paper_1805_12498_amd import build
        build.build()
