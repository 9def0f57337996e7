"""Build libdwa.so (gfx950) in-tree with hipcc.

    python -m paper_1501_04950_amd.build

Each source is compiled to an object in parallel (one translation unit per field
precision carries the site-local kernels, and one per precision and tile size the fused
hop), then linked into one shared library.  Device
code targets gfx950 only, with packed FP32 instructions turned off.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = ([f"csrc/kernels_hop_{p}_{ns}.hip" for p in ("f64", "f32", "bf16") for ns in (8, 16, 32)]
           + ["csrc/kernels_f64.hip", "csrc/kernels_f32.hip", "csrc/kernels_bf16.hip",
              "csrc/kernels.hip", "csrc/adjoint.hip", "csrc/scratch.hip", "csrc/api.cpp",
              "csrc/smat.cpp", "csrc/zolotarev.cpp"])
LIB = os.path.join(PKG, "libdwa.so")
OBJDIR = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(PKG, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops' is not a recognized feature" not in l and l.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    return obj, msgs


def build(verbose=True, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    for _, msgs in results:
        for m in msgs:
            print(m, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in results] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
