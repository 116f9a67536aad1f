import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers",
                            "gpu: runs on an MI355X through the HIP library's C-ABI")


@pytest.fixture(scope="session")
def oracle_ref():
    from oracle import ref
    ref._load()
    return ref
