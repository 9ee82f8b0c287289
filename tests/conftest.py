import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


@pytest.fixture
def rng():
    """A fresh seeded generator per test, so draws do not depend on test order."""
    import numpy as np
    return np.random.default_rng(12345)
