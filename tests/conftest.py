import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def small_wl():
    from synth import make_smallest
    return make_smallest()


@pytest.fixture(scope="session")
def small_oracle(small_wl):
    from oracle import rpa
    return rpa.solve_workload(small_wl, 0, return_all=True)


@pytest.fixture(scope="session")
def tiny():
    from synth import make_tiny
    return make_tiny()
