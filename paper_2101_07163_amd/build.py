"""Build libsnowlb.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "libsnowlb.so")
SOURCES = [os.path.join(HERE, "csrc", s) for s in ("snowlb_kernels.hip", "snowlb_io.hip", "snowlb_adjoint.hip",
                                                    "snowlb_api.cpp", "snowlb3d_kernels.hip", "snowlb3d_api.cpp")]
ARCH = os.environ.get("SNOWLB_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU instructions (the scalar and
# float2 code paths are used instead).
HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
