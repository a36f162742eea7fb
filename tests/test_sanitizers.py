"""The serial oracle under AddressSanitizer and UndefinedBehaviorSanitizer on
the CPU: tests/native/oracle_sanitize_main.c compiles the oracle source with
both sanitizers (no recovery) and assembles small seeded problems in every
mode the oracle has (both keyings, cap-region sampling, two other
strategies, an outer-tet subset, a polynomial g in the inner integrals),
checking A 1 = 0, symmetry and the CG along the way.  A sanitizer report ends
the run with a nonzero status."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import meshgen as mg
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "oracle_sanitize_main.c")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_san")
    cmd = [gcc, "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *SAN, "-o", exe, DRIVER, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr or "ubsan" in r.stderr or "sanitize" in r.stderr:
            pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
        raise AssertionError(r.stderr)
    return exe


def _case(pb, strategy=0, caps=0, keying=0, mask=None, g_coef=None, g_degree=-1):
    m = pb.mesh
    V, K = m.coords.shape[0], m.tets.shape[0]
    out = [struct.pack("<qqddiQiiiii", V, K, pb.delta, pb.psi, pb.mc_samples, pb.seed, strategy, caps, keying,
                       g_degree, 1 if mask is not None else 0)]
    out.append(np.ascontiguousarray(m.coords, dtype="<f8").tobytes())
    out.append(np.ascontiguousarray(m.tets, dtype="<i4").tobytes())
    out.append(np.ascontiguousarray(pb.vertex_free, dtype=np.uint8).tobytes())
    out.append(np.ascontiguousarray(pb.f_qp, dtype="<f8").reshape(K, 4).tobytes())
    out.append(np.ascontiguousarray(pb.g_nodal, dtype="<f8").reshape(V).tobytes())
    if mask is not None:
        out.append(np.ascontiguousarray(mask, dtype=np.uint8).tobytes())
    if g_coef is not None:
        out.append(np.ascontiguousarray(g_coef, dtype="<f8").tobytes())
    return b"".join(out)


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = _build(tmp_path)
    pb = mg.make_problem("san", 6, delta=0.25, jitter=0.15, jitter_seed=4, mc_samples=16, seed=3)
    K = pb.mesh.n_tets
    mask = mg.outer_subset_mask(K, 0.3, seed=7)
    # g = 1 + 2 x - y as tensor coefficients [a + 2 (b + 2 c)] of x^a y^b z^c
    coef = np.zeros(8)
    coef[0], coef[1], coef[2] = 1.0, 2.0, -1.0
    cases = [
        _case(pb),                                   # fullcaps, pair keying
        _case(pb, keying=1),                         # element keying
        _case(pb, caps=1),                           # caps sampled on E minus U_I
        _case(pb, strategy=oracle.STRATEGIES["nocaps"]),
        _case(pb, strategy=oracle.STRATEGIES["barycenter"]),
        _case(pb, mask=mask),                        # outer-tet subset
        _case(pb, g_coef=coef, g_degree=1),          # g itself in the inner integrals
    ]
    path = tmp_path / "cases.bin"
    path.write_bytes(b"".join(cases))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(path)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
    assert r.stdout.count("case ") == len(cases)
    assert "free=0 " not in r.stdout  # every case assembles free rows


def test_sanitizer_build_reports_a_heap_overflow(tmp_path):
    """The same compiler flags on a five-line program that reads past a heap
    block: the run must fail with an AddressSanitizer report, so a clean run
    of the oracle above means something."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    src = tmp_path / "overflow.c"
    src.write_text("#include <stdlib.h>\n"
                   "int main(int argc, char **argv) {\n"
                   "    int *a = malloc(4 * sizeof(int));\n"
                   "    int v = a[argc + 3];\n"
                   "    free(a);\n"
                   "    return v == 12345;\n"
                   "}\n")
    exe = str(tmp_path / "overflow")
    r = subprocess.run([gcc, "-O0", "-g", *SAN, "-o", exe, str(src)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr and "heap-buffer-overflow" in r.stderr


def test_hip_host_sanitizer_flags_report_undefined_behaviour(tmp_path):
    """The flags tests/native/build_host_sanitized.py gives hipcc (the
    sanitizer behind -Xarch_host, host code only) on a host-only program with
    a signed overflow: the run must fail with an UndefinedBehaviorSanitizer
    report, so the clean GPU run of the library's host code means something."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("build_host_sanitized",
                                                  os.path.join(HERE, "native", "build_host_sanitized.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not os.path.exists(mod.libbuild.HIPCC):
        pytest.skip("no hipcc")
    src = tmp_path / "overflow.hip"
    src.write_text("#include <hip/hip_runtime.h>\n"
                   "#include <climits>\n"
                   "int main(int argc, char **argv) {\n"
                   "    int v = INT_MAX - 1 + argc;\n"
                   "    v += argc;\n"
                   "    return v == 7;\n"
                   "}\n")
    exe = str(tmp_path / "overflow")
    r = subprocess.run([mod.libbuild.HIPCC, *mod.libbuild.FLAGS, *mod.HOST_SAN, "-o", exe, str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60,
                       env=dict(os.environ, UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode != 0
    assert "runtime error" in r.stderr and "overflow" in r.stderr, r.stderr[-2000:]
