"""Build libshatterbc.so for gfx950 in-tree (paper_1209_6007_amd/libshatterbc.so).

Host-only C++ is compiled with g++, HIP sources with hipcc for gfx950, and the
objects are linked by hipcc into one shared library.  Usable as a module
(``build()``) or a script (``python build.py [--jobs N]``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libshatterbc.so")
OBJ = os.path.join(ROOT, "_build", "obj")

HOST_SOURCES = ["prep.cpp", "far.cpp"]
HIP_SOURCES = ["kernels.hip", "runtime.hip", "api.hip", "server.hip", "noalloc.hip", "far_api.hip"]

ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # packed FP32 instructions stay off: they are not needed here and some of
    # their forms are unreliable on the target parts
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    return out


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()
    cmds = []
    objs = []
    for s in HOST_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        cmds.append(["g++", *HOST_FLAGS, f"-I{INCLUDE}", "-c", os.path.join(HERE, s), "-o", o])
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        cmds.append([hipcc, *HIP_FLAGS, f"-I{INCLUDE}", "-c", os.path.join(HERE, s), "-o", o])
        objs.append(o)
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, OUT)
    build_c_tests(hipcc)
    return OUT


C_TESTS = [("tests/c_api/device_path.cpp", "tests/c_api/device_path"), ("tests/c_api/noalloc.cpp", "tests/c_api/noalloc")]


def build_c_tests(hipcc: str) -> None:
    """Small C++ consumers of the public header, linked against the library."""
    for src, exe in C_TESTS:
        s = os.path.join(ROOT, src)
        if not os.path.exists(s):
            continue
        out = os.path.join(ROOT, exe)
        _run([hipcc, f"--offload-arch={ARCH}", "-O2", "-std=c++17", f"-I{INCLUDE}", s, "-o", out + ".tmp",
              f"-L{PKG}", "-lshatterbc", f"-Wl,-rpath,{PKG}", "-Wl,-rpath,$ORIGIN/../../paper_1209_6007_amd"])
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    j = None
    if "--jobs" in sys.argv:
        j = int(sys.argv[sys.argv.index("--jobs") + 1])
    print(build(jobs=j, verbose="-v" in sys.argv))
