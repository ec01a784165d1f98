"""Build libsakura.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsakura.so")
SOURCES = [os.path.join(CSRC, "sakura.hip"), os.path.join(CSRC, "batch.hip"),
           os.path.join(CSRC, "guess.hip")]
HEADERS = [os.path.join(CSRC, "kepler_device.hpp"), os.path.join(CSRC, "common.hpp"),
           os.path.join(CSRC, "guess_device.hpp"), os.path.join(CSRC, "tiles.hpp"),
           os.path.join(os.path.dirname(HERE), "include", "sakura.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + HIPCC_FLAGS + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
