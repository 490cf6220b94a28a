import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# Load the HIP library before torch: it then binds to the ROCm runtime it was
# built against instead of the older copy bundled with torch (both carry the
# same soname, and the first one loaded serves the whole process).
try:
    import paper_1209_6007_amd as _sbc

    _sbc.lib()
except Exception:  # pragma: no cover - a missing build is reported by the tests themselves
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests are selected with -m gpu; without a visible GPU they are skipped
    # rather than failing, so `-m "not gpu"` and a bare run both work on CPU.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
