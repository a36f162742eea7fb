"""Builds libnlfem.so (HIP, gfx950) in-tree from csrc/*.hip."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnlfem.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("NLFEM_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # bit-reproducible floating point: no implicit contraction, IEEE sqrt/div
         "-ffp-contract=off",
         # no packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = ["k_sort.hip", "k_plan.hip", "k_numeric.hip", "k_rows.hip", "k_cg.hip", "runtime.hip", "capi.hip", "server.hip"]
EXTRA = os.environ.get("NLFEM_EXTRA_FLAGS", "").split()


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA, "-c", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(verbose: bool = False, out_lib: str | None = None, build_dir: str | None = None) -> str:
    global OUT
    lib = out_lib or LIB
    if build_dir:
        OUT = build_dir
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
