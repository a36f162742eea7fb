"""The library's host code under UndefinedBehaviorSanitizer:
tests/native/_build/nlfem_host_sanitized (built by __graft_entry__.build()
through tests/native/build_host_sanitized.py; the sanitizer is in the host
code only, the GPU code is the ordinary build) drives plans in four modes with
assembly and plan CG, a mesh error, a batch built on the builder threads and
a failing one, and the server's worker threads, all through the C ABI.  A
sanitizer report, or a failed check, ends it with a nonzero status.
(AddressSanitizer's ROCm runtime stops on an internal check of its
device-allocator hook at the first HIP call on GPUs without XNACK, so it
covers the oracle on the CPU instead.)"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "native", "_build", "nlfem_host_sanitized")


def test_host_code_under_undefined_behaviour_sanitizer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.skip("the host-sanitized driver is not built (__graft_entry__.build() builds it)")
    sys.stdout.write("[gpu-test] host-sanitized driver\n")
    sys.stdout.flush()
    env = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=280, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
