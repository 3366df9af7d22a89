import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "exhaustive: all 2^32 float32 patterns (set LLAMA_EXHAUSTIVE=1)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LLAMA_EXHAUSTIVE") == "1":
        return
    skip = pytest.mark.skip(reason="exhaustive 2^32 sweep: set LLAMA_EXHAUSTIVE=1")
    for it in items:
        if "exhaustive" in it.keywords:
            it.add_marker(skip)
