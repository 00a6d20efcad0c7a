import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


@pytest.fixture(scope="session")
def tiny():
    import synth
    return synth.workload_tiny()


@pytest.fixture(scope="session")
def small_body():
    """Human-like template with 3,000 vertices on a 160x120 camera."""
    import synth
    cam = dict(width=160, height=120, fx=131.25, fy=131.25, cx=79.5, cy=59.5)
    return synth.make_body(3000, cam, 2.6)


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(1234)
