"""The library's own sources built for the CPU against a HIP emulation
(tests/cpu_emu) and run under AddressSanitizer: kernel indexing, slot sizing,
queue handling and error paths are checked against the oracle without a GPU.

The emulated runtime starts device memory and LDS with garbage and leaves a
sticky error behind from a failing device query, as a real runtime can; the
library must neither read before writing nor mistake a stale error for a
failed launch (an early return used to free buffers under a running kernel).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def emu_lib():
    if not _asan():
        pytest.skip("libasan not available")
    sys.path.insert(0, os.path.join(ROOT, "tests", "cpu_emu"))
    from tests.cpu_emu import build_emu

    return build_emu.build(asan=True)


CHECKS = ["single", "pieces", "whole", "hubs", "team", "wave", "noalloc", "server", "far"]


@pytest.fixture(scope="module")
def runs(emu_lib):
    """All check groups start at once, each in its own process."""
    env = dict(os.environ)
    env["LD_PRELOAD"] = _asan()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    procs = {w: subprocess.Popen([sys.executable, os.path.join(ROOT, "tests", "cpu_emu", "run_checks.py"), w],
                                 cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for w in CHECKS}
    yield procs
    for p in procs.values():
        if p.poll() is None:
            p.kill()
            p.wait()


@pytest.mark.parametrize("which", CHECKS)
def test_emulated_library(runs, which):
    p = runs[which]
    out, _ = p.communicate(timeout=1200)
    assert p.returncode == 0 and "ALL OK" in out, out[-4000:]
