import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

import pytest  # noqa: E402


def pytest_collection_modifyitems(config, items):
    # a GPU test collected on a machine without a GPU is reported as skipped
    # only when the marker is deselected; nothing to do here otherwise
    return


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.load()
