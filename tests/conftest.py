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
def cfg1():
    from synth import make_config1
    return make_config1()


@pytest.fixture(scope="session")
def cfg1_oracle(cfg1):
    from oracle import rpa
    return rpa.solve_workload(cfg1, 0, return_all=True)


@pytest.fixture(scope="session")
def tiny():
    from synth import make_tiny
    return make_tiny()
