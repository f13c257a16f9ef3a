import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size parity case (minutes of host work)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture
def substitution():
    """Run the test with the sweeps' diagonal blocks solved by substitution
    (exact on exactly representable data) instead of by their inverses."""
    import paper_2601_14466_amd as mg
    h = mg.handle()
    h.set_solve_mode("substitution")
    yield h
    h.set_solve_mode("inverse")
