import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the GPU)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def _ensure_built():
    import gsp_inputs
    import oracle
    if not os.path.exists(gsp_inputs._LIB_PATH):
        gsp_inputs.build()
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()


_ensure_built()
