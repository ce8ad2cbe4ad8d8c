import importlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    ob = importlib.import_module("oracle.build")
    src = os.path.join(os.path.dirname(ob.LIB), "oracle.c")
    if not os.path.exists(ob.LIB) or os.path.getmtime(src) > os.path.getmtime(ob.LIB):
        ob.build()
