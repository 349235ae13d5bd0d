import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; calls the HIP library through the C-ABI")
    config.addinivalue_line("markers", "slow: long CPU-only oracle run")


def pytest_collection_modifyitems(config, items):
    # Tests marked slow are skipped unless CASCLB_SLOW=1 is set.
    if os.environ.get("CASCLB_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle run; set CASCLB_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
