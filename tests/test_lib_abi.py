"""CPU-side checks of the C ABI library: it is built, loads, exports every
entry point that include/nlfem.h declares, and reports the device error when
no GPU is present.  No compute calls are made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlfem.h")


def _declared():
    txt = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)  # declarations only, not comments
    return sorted(set(re.findall(r"\b(nlfem_[a-z_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for need in ["nlfem_create", "nlfem_plan_create", "nlfem_assemble", "nlfem_cg", "nlfem_plan_destroy",
                 "nlfem_debug_pairs", "nlfem_plan_info"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2302_07499_amd as P
    L = P.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(P.EXPORTS) >= set(_declared())


def test_rule_constants_match_oracle(orc):
    import paper_2302_07499_amd as P
    assert P.nlfem_rule_constants() == orc.rule_constants()


def test_null_and_no_device_errors():
    import torch
    import paper_2302_07499_amd as P
    L = P.load()
    assert L.nlfem_create(None, 0, None, 0) == P.NLFEM_E_INVALID_ARG
    assert L.nlfem_plan_create(None, None, None, None) == P.NLFEM_E_INVALID_ARG
    assert L.nlfem_plan_destroy(None) == P.NLFEM_E_INVALID_ARG
    if not torch.cuda.is_available():
        ctx = C.c_void_p()
        assert L.nlfem_create(C.byref(ctx), 0, None, 0) == P.NLFEM_E_DEVICE


def test_server_null_and_no_device_errors():
    import torch
    import paper_2302_07499_amd as P
    L = P.load()
    assert L.nlfem_server_create(0, 4, 0, None) == P.NLFEM_E_INVALID_ARG
    h = C.c_void_p()
    assert L.nlfem_server_create(0, 0, 0, C.byref(h)) == P.NLFEM_E_INVALID_ARG
    assert L.nlfem_server_submit(None, None, None, None, None, None, None) == P.NLFEM_E_INVALID_ARG
    assert L.nlfem_server_poll(None, 1, None) == P.NLFEM_E_INVALID_ARG
    assert L.nlfem_server_destroy(None) == P.NLFEM_E_INVALID_ARG
    if not torch.cuda.is_available():
        assert L.nlfem_server_create(0, 2, 1 << 20, C.byref(h)) == P.NLFEM_E_DEVICE
