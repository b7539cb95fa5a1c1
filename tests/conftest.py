import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """The oracle and the generator are host code: build them if absent."""
    import synth
    from oracle import oracle

    if not os.path.exists(synth.LIB):
        synth.build()
    if not os.path.exists(oracle.LIB):
        oracle.build()
    yield
