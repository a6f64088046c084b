"""Build libgz.so (host C++ and HIP kernels for gfx950) in-tree with hipcc.

Usage: ``python -m paper_1911_12877_amd.build``.  The library is written to
``paper_1911_12877_amd/_build/libgz.so``.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(OUT_DIR, "libgz.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["graph_prep.cpp", "compiler.cpp", "capi.cpp", "learned.cpp", "mine.hip", "mlp.hip",
           "prep.hip"]

# gfx950 only; packed FP32 instructions are switched off for every HIP
# translation unit (the library uses no floating point on the device, the
# flag keeps it that way for future code).
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    cmds = []
    incs = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT_DIR, src + ".o")
        cmd = [HIPCC] + HIP_FLAGS + incs + ["-c", path, "-o", obj]
        if src.endswith(".cpp"):
            # host-only translation units: plain g++ against the HIP headers
            cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-Wall",
                   "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"] + \
                incs + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # translation units compile independently; the largest first
    order = sorted(range(len(cmds)), key=lambda i: -os.path.getsize(
        os.path.join(CSRC, SOURCES[i])))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as pool:
        for f in [pool.submit(subprocess.check_call, cmds[i]) for i in order]:
            f.result()
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
