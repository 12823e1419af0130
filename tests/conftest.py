import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


@pytest.fixture(scope="session")
def shale8192():
    """The fractured-shale medium at its full 8192 x 8192 size (seed 3),
    generated once per session."""
    from paper_1411_7051_amd import inputs
    return inputs.shale(n=8192, seed=3)
