"""Build libqtt.so (HIP kernels + C ABI) for gfx950 with hipcc.

Run as ``python -m paper_2501_07778_amd.build`` or call ``build()``.  Every
source is compiled to an object under ``_build/`` and linked into
``paper_2501_07778_amd/libqtt.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqtt.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("QTT_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "capi.cpp",
    "assemble.cpp",
    "solve.cpp",
    "als.cpp",
    "k_tt.hip",
    "k_round.hip",
    "k_sketch.hip",
    "k_als.hip",
    "k_full.hip",
    "batched.cpp",
    "graph.cpp",
    "k_mlp.hip",
    "noalloc.cpp",
    "ktimer.cpp",
    "combine.cpp",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "--offload-arch=" + ARCH,
    # packed FP32 instructions stay off for every device pass
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
