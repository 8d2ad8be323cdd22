import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU-side oracle run")


def pytest_sessionstart(session):
    """Build the HIP library and the C oracle only when they are missing (a fresh checkout)."""
    from paper_1812_10302_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1812_10302_amd import build as hip_build
        hip_build.build()
    from oracle.cascade import cascade_path, build_cascade
    if not os.path.exists(cascade_path()):
        build_cascade()
