import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libsgml.so")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    # the oracle is C; build it once per session if missing or stale
    from oracle import build
    if not os.path.exists(build.LIB) or os.path.getmtime(build.LIB) < os.path.getmtime(build.SRC):
        build.build()
