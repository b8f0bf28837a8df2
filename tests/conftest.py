"""pytest configuration: markers and shared helpers.

Markers
  gpu   needs an MI355X (gfx950) and the built HIP library; run with -m gpu
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")

