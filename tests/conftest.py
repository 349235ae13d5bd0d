import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; calls the HIP library through the C-ABI")
    config.addinivalue_line("markers", "slow: long CPU-only oracle run")
    # PyTorch ships its own HIP runtime beside the ROCm one the library links.
    # PyTorch finds the GPU only if its runtime initialises first, so when GPU
    # tests may run (they use PyTorch for device memory), initialise it before
    # any test module touches the library.
    markexpr = (config.getoption("markexpr", default="") or "").replace(" ", "")
    if markexpr != "notgpu":
        try:
            import torch

            torch.cuda.is_available()
        except Exception:
            pass


def pytest_collection_modifyitems(config, items):
    # Tests marked slow are skipped unless CASCLB_SLOW=1 is set.
    if os.environ.get("CASCLB_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle run; set CASCLB_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
