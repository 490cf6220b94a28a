import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# The GPU tests talk to the library only (no torch in this process): the
# library binds the ROCm runtime it was built against, and torch, which
# bundles an older copy of the same libraries, would otherwise mix the two.
_LIB_OK = False
_HAVE_GPU = False
try:
    import paper_1209_6007_amd as _sbc

    _sbc.lib()
    _LIB_OK = True
    try:
        _c = _sbc.Context(0)
        _c.close()
        _HAVE_GPU = True
    except Exception:
        _HAVE_GPU = False
except Exception:  # a missing build: GPU tests then fail loudly instead of being skipped
    _LIB_OK = False


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    if _HAVE_GPU or not _LIB_OK:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
