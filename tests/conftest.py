import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long test: 10^8-draw statistics, or every output of a 2^28-2^30 fill")


@pytest.fixture(scope="session")
def O():
    from oracle import oracle
    oracle.build()
    return oracle
