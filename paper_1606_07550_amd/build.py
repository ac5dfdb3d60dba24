"""Build the native libraries in-tree.

* ``libtricc.so``: the gfx950 HIP kernels and the C ABI declared in
  ``include/tricc.h`` (hipcc, one object per source, then linked).
* ``inputs/libtricc_gen.so``: the seeded input generators (g++).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libtricc.so")
ARCH = os.environ.get("TRICC_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["api.hip", "build_kernels.hip", "clique_kernels.hip", "core_kernels.hip", "count_kernels.hip",
               "gen_kernels.hip", "query_kernels.hip", "serve_kernels.hip", "serve_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = (r.stdout + r.stderr).strip()
    # hipcc's host pass does not know the GPU target feature; that note is noise
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines), flush=True)


def build_hip(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in HIP_SOURCES]
    cmds = [[HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(HIP_SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    _run([HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", *objs, "-o", LIB + ".tmp"], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build(verbose=False):
    from .inputs import build as build_gen
    build_gen(verbose)
    return build_hip(verbose)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_1606_07550_amd.build import build as _b
    print(_b(verbose=True))
