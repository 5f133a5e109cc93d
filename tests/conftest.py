import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long physics run, only with LBM_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LBM_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="long physics run; set LBM_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
