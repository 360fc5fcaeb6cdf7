import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); runs through the C-ABI")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import lbref
    lbref.build()
    for v in lbref.VARIANTS:
        lbref.build(variant=v)
    yield
