import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    import oracle
    # the oracle's OpenMP threads: the host's cores, at most 16 (a GPU host's share per GPU)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield
