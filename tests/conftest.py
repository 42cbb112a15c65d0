import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def small_elasticity():
    import fegen
    import oracle
    prob, b = fegen.elasticity_small(N=32)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    return prob, b, h
