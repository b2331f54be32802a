"""Build liblrx.so (HIP kernels + C ABI) for gfx950 with hipcc.

Each translation unit is compiled in parallel into ``_build/`` and linked
in-tree as ``paper_2602_05255_amd/liblrx.so``.  Run ``python -m
paper_2602_05255_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblrx.so")

# (source, object name, extra flags); the determinant kernels build once per bulk dtype.
SOURCES = [("lrx_capi.cpp", "lrx_capi", []), ("lrx_pf.hip", "lrx_pf", []), ("lrx_flush.hip", "lrx_flush", []),
           ("lrx_factor.hip", "lrx_factor", []), ("lrx_adjoint.hip", "lrx_adjoint", []),
           ("lrx_window.hip", "lrx_window", []), ("lrx_general.hip", "lrx_general", []),
           ("lrx_pf_fused.hip", "lrx_pf_fused", [])] + \
          [("lrx_det.hip", f"lrx_det_{i}", [f"-DLRX_DT={i}"]) for i in range(4)]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # Packed FP32 instructions are kept out of the generated code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _compile(item) -> str:
    src, name, extra = item
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
