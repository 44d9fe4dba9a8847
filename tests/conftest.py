import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def met_c1():
    import inputs
    return inputs.make_met_c1(seed=11)


@pytest.fixture(scope="session")
def orc_c1(met_c1):
    import oracle
    return oracle.Met(met_c1)


@pytest.fixture()
def rng():
    return np.random.Generator(np.random.PCG64(1234))
