import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: longer CPU test (still part of the CPU suite)")


@pytest.fixture(scope="session")
def sphere16():
    """Oracle fractions and operators of the 16^3 sphere (R = 0.45, sigma = 5)."""
    from oracle import geometry as geo, operators as ops
    n = (16, 16, 16)
    h = 1.0 / 16
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    return fr, ops.build(fr, n, h, 5.0)
