import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long run (minutes of oracle time), collected only with LB_SLOW_TESTS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LB_SLOW_TESTS") == "1":
        return
    skip = pytest.mark.skip(reason="long run: set LB_SLOW_TESTS=1 to include it")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    import oracle
    # the oracle's OpenMP threads: the host's cores, at most 16 (a GPU host's share per GPU)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield
