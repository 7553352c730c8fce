import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")


@pytest.fixture(scope="session")
def oracle_pool():
    """Worker processes for long oracle replays (spawned; NumPy and the oracle only)."""
    from tests.parity import replay_pool

    pool = replay_pool()
    yield pool
    pool.shutdown(wait=True, cancel_futures=True)
