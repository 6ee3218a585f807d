import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size (up to 2e9 points) checks")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """Compile the host-only C libraries (generators, oracle) if they are not built."""
    import oracle
    import synth

    synth.build(force=False)
    oracle.build(force=False)
