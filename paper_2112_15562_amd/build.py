"""Build ``libbttb.so`` (the HIP library behind the C ABI in ``include/bttb.h``) for gfx950.

Usage: ``python paper_2112_15562_amd/build.py``.  Each source is compiled with hipcc in
parallel, then linked into the package directory, where the binding loads it from.
This file imports nothing from the package, so it can run before the library exists.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbttb.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["operator.hip", "operator_fast.hip", "group.hip", "group_mixed_f32.hip", "group_mixed_f64.hip",
           "autotune.hip", "prism.hip", "rrcg.hip", "rrcg_group.hip", "noalloc.hip", "status.cpp"]
HEADERS = ["common.h", "fft_engine.h", "fft_reg.h", "fast_kernels.h", "rrcg_fuse.h", "rrcg_kernels.h", "group.h",
           "group_kernels.h", "group_mixed.h"]

ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fvisibility=hidden",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libbttb.so; returns the library path."""
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def is_built() -> bool:
    return os.path.exists(LIB)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
