import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def built_lib():
    """Path of libdsbt.so, building it in-tree (hipcc cross-compiles for gfx950) if missing."""
    from paper_1509_07115_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1509_07115_amd import build
        build.build()
    return _lib.LIB_PATH
