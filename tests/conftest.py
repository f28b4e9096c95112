import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_collection_modifyitems(config, items):
    # slow tests (the FP64 oracle runs for minutes) only with PM_RUN_SLOW=1
    if os.environ.get("PM_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle run; set PM_RUN_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")
