"""Build libdpmi.so (the HIP library behind include/dpmi.h) for gfx950.

hipcc compiles each source to an object in parallel, then links the shared
library in the package directory, where the Python binding loads it.
The neighbour-list source is compiled with -ffp-contract=off so that pair
distances are bit-reproducible; every HIP source gets the packed-FP32
feature switched off.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdpmi.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["api.cpp", "k_nlist.hip", "k_env.hip", "k_embed_f64.hip", "k_fit_f64.hip", "k_md.hip",
           "k_embed_mix.hip", "k_embed_wide.hip", "k_fit_mix.hip", "k_student.hip"]
EXACT_FP = {"k_nlist.hip"}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags(src):
    f = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fno-gpu-rdc",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-mllvm", "-amdgpu-mfma-vgpr-form", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-I", INCLUDE, "-I", CSRC]
    if src in EXACT_FP:
        f.append("-ffp-contract=off")
    return f


def build(verbose=False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()

    def one(src):
        obj = os.path.join(BUILD, src + ".o")
        cmd = [cc, *_flags(src), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
