import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X")
    config.addinivalue_line("markers", "slow: long CPU test")
    # the oracle's results do not depend on its thread count: use the host's cores
    import oracle
    oracle.set_threads(min(16, os.cpu_count() or 1))


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
