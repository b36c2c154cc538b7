import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test (still part of the CPU suite)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


def announce(*parts):
    """Names the case on stdout before a GPU step, so a crash still shows it."""
    print("[case]", *parts, flush=True)
