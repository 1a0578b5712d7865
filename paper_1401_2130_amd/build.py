"""Build ``libperc.so`` (the C-ABI library of include/perc.h) for gfx950 with hipcc.

Run ``python paper_1401_2130_amd/build.py`` (or ``__graft_entry__.build()``); the
script does not import the package, so it works while the library is missing. The
library lands in ``paper_1401_2130_amd/_build/libperc.so``, in-tree, so that it ships
with the source tree to the machine that runs it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(OUT_DIR, "libperc.so")
SOURCES = ["kernels.hip", "lattice.cpp", "perc_api.cpp"]
ARCH = os.environ.get("PERC_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


# device code: packed FP32 instructions stay off (the compiler must not form them), and
# FP32 denormals are kept: a reached tube's state word never drops below the smallest
# denormal, which is how the kernels carry the exact reached set
_DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-fno-gpu-flush-denormals-to-zero"]
_HOST_FLAGS = ["-x", "c++", f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__=1"]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        cmd[1:1] = _DEVICE_FLAGS if src.endswith(".hip") else _HOST_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libperc.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
