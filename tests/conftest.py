import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    from oracle import build as ob
    if not os.path.exists(oracle.LIB_PATH):
        ob.build()
    return True


def pytest_collection_modifyitems(config, items):
    # GPU tests import torch lazily; nothing to change here beyond the marker
    return None
