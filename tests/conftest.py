import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _ensure_oracle():
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()


_ensure_oracle()


@pytest.fixture(scope="session")
def root():
    return ROOT
