"""Build the library's own sources for the CPU against the HIP emulation in
tests/cpu_emu/hip -- TEST INFRASTRUCTURE.  The result, libshatterbc_emu.so, is
instrumented with AddressSanitizer and is only ever loaded by the emulation
checks; the product loads nothing but the gfx950 build."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1209_6007_amd", "csrc")
OUT_DIR = os.path.join(ROOT, "_build", "emu")
OUT = os.path.join(OUT_DIR, "libshatterbc_emu.so")
SOURCES = ["prep.cpp", "far.cpp", "kernels.hip", "runtime.hip", "api.hip", "server.hip", "noalloc.hip", "far_api.hip"]


def build(asan: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-fno-omit-frame-pointer", "-Wno-unused-function",
             "-DSBC_EMU_FEW_VARIANTS=1", f"-I{HERE}",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    if asan:
        flags.append("-fsanitize=address")
    objs = [os.path.join(OUT_DIR, s + ".o") for s in SOURCES]

    def compile_one(k):
        subprocess.check_call(["g++", *flags, "-c", "-x", "c++", os.path.join(CSRC, SOURCES[k]), "-o", objs[k]])

    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(compile_one, range(len(SOURCES))))
    tmp = OUT + ".tmp"
    subprocess.check_call(["g++", *flags, "-shared", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(asan="--no-asan" not in sys.argv))
