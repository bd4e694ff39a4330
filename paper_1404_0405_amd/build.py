"""Compile the HIP library ``libwt.so`` for gfx950 in-tree (hipcc cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libwt.so")

SOURCES = ["wt_grid.cpp", "wt_pair.cpp", "wt_lattice.cpp", "wt_api.cpp", "wt_mlp_api.cpp", "wt_alloc.cpp", "wt_kernels.hip",
           "wt_ml.hip", "wt_lattice.hip", "wt_mlp.hip", "wt_learn.hip", "wt_compact.hip", "wt_batch.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", f"-I{ROOT}/include"]
HIP_FLAGS = ["--offload-arch=gfx950", "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]
# per-source extra flags: the lattice kernel holds its tile geometry in registers and prefetches
# the next lozenge; the iterative ILP scheduler keeps it within 256 VGPRs without spilling
# (a spill reload would make the kernel wait for the prefetch)
EXTRA = {"wt_lattice.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(src):
    out = os.path.join(OBJ, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    cmd = [_hipcc(), *COMMON]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", *HIP_FLAGS]
    cmd += EXTRA.get(src, [])
    cmd += ["-c", path, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
