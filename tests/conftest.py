import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    # GPU tests import torch lazily; make sure that when they run, torch (and its
    # HIP runtime) is loaded before the library so both share one runtime.
    if any("gpu" in item.keywords for item in items):
        try:
            import torch  # noqa: F401
        except Exception:
            pass


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle._load()
    return oracle
