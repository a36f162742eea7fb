"""nlfem_cg_noalloc, the CG entry point for callers that cannot allocate
device memory: its work vectors live in the library's static device scratch.
Checked against nlfem_cg on the same systems (bitwise: the same kernels in the
same order), on two calls in a row, the second with a smaller system, and the
size limit is rejected with a clear error."""
import sys

import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write(f"[gpu-test] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_07499_amd as P
    d = P.Device(0)
    yield d
    d.close()


def _system(dev, pb):
    plan = dev.plan_problem(pb)
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    return plan, s


def _both(dev, s):
    import paper_2302_07499_amd as P
    t = dev.torch
    xa = t.zeros(s.n_free, dtype=t.float64, device=dev.dev)
    xb = t.full((s.n_free,), 7.0, dtype=t.float64, device=dev.dev)
    xb.zero_()
    ita, rra, oka = P.nlfem_cg(dev.ctx, s.n_free, s.ff_row_ptr, s.ff_col, s.ff_val, s.rhs, xa, 1e-10)
    itb, rrb, okb = P.nlfem_cg_noalloc(dev.ctx, s.n_free, s.ff_row_ptr, s.ff_col, s.ff_val, s.rhs, xb, 1e-10)
    return (xa, ita, rra, oka), (xb, itb, rrb, okb)


def test_noalloc_cg_equals_cg_twice_then_smaller(dev):
    import paper_2302_07499_amd as P
    big = mg.make_problem("noalloc-big", 12, delta_over_h=2.0, jitter=0.15, seed=3, mc_samples=16)
    small = mg.plain_problem()
    sizes = []
    for name, pb in [("big", big), ("small", small)]:
        _say(f"no-alloc CG on {name} (n = {pb.mesh.n_tets} tets)")
        plan, s = _system(dev, pb)
        (xa, ita, rra, oka), (xb, itb, rrb, okb) = _both(dev, s)
        _say(f"  n_free {s.n_free}: cg {ita} it {rra:.3e}, noalloc {itb} it {rrb:.3e}")
        assert oka and okb and ita == itb and rra == rrb
        assert dev.torch.equal(xa, xb)
        sizes.append(s.n_free)
        plan.destroy()
    assert sizes[1] < sizes[0]


def test_noalloc_cg_rejects_oversized_system(dev):
    import ctypes as C
    import paper_2302_07499_amd as P
    L = P.load()
    it, rr = C.c_int32(), C.c_double()
    one = C.c_void_p(1)  # never dereferenced: the size check comes first
    n = (1 << 19) + 1
    st = L.nlfem_cg_noalloc(dev.ctx, n, one, one, one, one, one, 1e-10, 10, C.byref(it), C.byref(rr))
    assert st == P.NLFEM_E_UNSUPPORTED
    assert "exceeds" in P.last_error(dev.ctx)
