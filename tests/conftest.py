import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # a test module under tests/ whose name starts with test_gpu_ is GPU-only by construction
    for it in items:
        if os.path.basename(str(it.fspath)).startswith("test_gpu_"):
            it.add_marker(pytest.mark.gpu)
