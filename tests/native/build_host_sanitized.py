"""Builds tests/native/_build/nlfem_host_sanitized: the library's sources with
UndefinedBehaviorSanitizer in the host code only (each sanitizer flag behind
-Xarch_host; the GPU code is built as usual), linked with
lib_sanitize_main.cpp.  AddressSanitizer is left out here: its ROCm runtime
hooks the HIP runtime's device allocator and stops on an internal check at the
first HIP call on GPUs run without XNACK (the oracle gets it on the CPU, in
tests/test_sanitizers.py).  Test infrastructure, run by
__graft_entry__.build() so that the GPU test finds it built."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_2302_07499_amd import build as libbuild  # noqa: E402

OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "nlfem_host_sanitized")
HOST_SAN = []
for f in ["-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]:
    HOST_SAN += ["-Xarch_host", f]


def _compile(src: str, obj: str, extra: list[str]) -> None:
    cmd = [libbuild.HIPCC, *libbuild.FLAGS, *HOST_SAN, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = [(os.path.join(libbuild.SRC, s), os.path.join(OUT, os.path.splitext(s)[0] + ".o"), [])
            for s in libbuild.SOURCES]
    jobs.append((os.path.join(HERE, "lib_sanitize_main.cpp"), os.path.join(OUT, "lib_sanitize_main.o"),
                 ["-x", "hip", "-I", os.path.join(ROOT, "include")]))
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        list(ex.map(lambda j: _compile(*j), jobs))
    tmp = EXE + ".tmp"
    cmd = [libbuild.HIPCC, f"--offload-arch={libbuild.ARCH}", *HOST_SAN, "-o", tmp, *[j[1] for j in jobs]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, EXE)
    if verbose:
        print("built", EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
