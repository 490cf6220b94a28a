"""GPU: the entry point that allocates no device memory
(sbc_piece_bc_noalloc), called through the C interface from a C++ program
that owns the device buffers: two calls in a row, the second on a smaller
piece, each equal to sbc_piece_bc to 1e-9 relative with device flags 0, and a
piece beyond SBC_NOALLOC_MAX_VERTICES refused."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_noalloc_entry_point_matches_piece_bc():
    exe = os.path.join(ROOT, "tests", "c_api", "noalloc")
    assert os.path.exists(exe), "build the C test programs with __graft_entry__.build()"
    r = subprocess.run([exe], cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0 and "noalloc ok" in r.stdout, r.stdout[-2000:]
