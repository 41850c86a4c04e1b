"""Compile the HIP library librcell.so for gfx950 (in-tree, with hipcc)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librcell.so")
SOURCES = ["rcell_md.hip", "rsur.hip", "rcell_probe.hip"]
HEADERS = ["md_device.h", "rsur_device.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    # roctx ranges around the API calls and the phases they enqueue
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check compiles every time it is called)."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *FLAGS, "-I", os.path.join(ROOT, "include"), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
