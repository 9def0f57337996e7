"""Build libdwa.so (gfx950) in-tree with hipcc.

    python -m paper_1501_04950_amd.build

Every source is compiled for gfx950 only, with packed FP32 instructions turned
off in device code.
"""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = ["csrc/kernels.hip", "csrc/api.cpp", "csrc/smat.cpp"]
LIB = os.path.join(PKG, "libdwa.so")


def hipcc_cmd(out=LIB):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return ([hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-x", "hip"]
            + [os.path.join(PKG, s) for s in SOURCES] + ["-o", out])


def build(verbose=True):
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
