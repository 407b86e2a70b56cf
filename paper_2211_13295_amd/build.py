"""Build the gfx950 HIP library libhog.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhog.so")
SOURCES = [os.path.join(HERE, "csrc", "hog.hip")]
HEADERS = [os.path.join(HERE, "csrc", f)
           for f in ("hog_kernels.h", "hog_physics.h", "hog_tables.h", "hog_gate.h", "hog_o2.h", "hog_rk.h", "hog_char.h")] + [
    os.path.join(ROOT, "include", "hog.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the gfx950 code (the device pass
    # honours the feature; the host pass warns that it does not know it)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in ordinary VGPRs: the gate and training kernels feed them
    # to VALU instructions, which would otherwise copy them out of AGPRs
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, extra=()):
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
