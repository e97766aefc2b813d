"""Build libpitsbicg.so in-tree with hipcc for gfx950.

Usage: python -m paper_2203_10148_amd.build   (or call build()).
Objects go to paper_2203_10148_amd/_build/, the library to
paper_2203_10148_amd/libpitsbicg.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpitsbicg.so")
# the checking build (-DPIT_CHECK: LDS poisoned with NaN before first use)
OBJ_CHECK = os.path.join(PKG, "_build_check")
LIB_CHECK = os.path.join(PKG, "libpitsbicg_check.so")
ARCH = os.environ.get("PIT_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, check: bool = False) -> str:
    obj = os.path.join(OBJ_CHECK if check else OBJ, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *COMMON, *(["-DPIT_CHECK"] if check else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def sources() -> list:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, jobs: int | None = None, check: bool = False) -> str:
    """Compile every HIP/C++ source and link libpitsbicg.so (always rebuilds);
    check=True builds libpitsbicg_check.so with -DPIT_CHECK instead."""
    odir, lib = (OBJ_CHECK, LIB_CHECK) if check else (OBJ, LIB)
    os.makedirs(odir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4) // 2), 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, check), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    build(verbose=True, check=True)
    sys.exit(0)
