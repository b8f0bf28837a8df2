"""pytest configuration: markers and shared helpers.

Markers
  gpu   needs an MI355X (gfx950) and the built HIP library; run with -m gpu
  slow  long CPU runs (oracle convergence studies); skipped unless
        VANSE_SLOW=1 is set in the environment
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run, enabled by VANSE_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("VANSE_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow: set VANSE_SLOW=1 to run")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
