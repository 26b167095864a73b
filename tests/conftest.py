import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large-size GPU case")


def pytest_collection_modifyitems(config, items):
    # GPU tests that run without a device fail loudly inside the test (the
    # library refuses to run without one); they are only deselected by -m.
    pass
