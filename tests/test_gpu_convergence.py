"""Convergence workload on the GPU (the paper's 3D accuracy experiment,
Sec. 5: Omega = (0,1)^3, delta = 0.1, u = prod x_d (1 - x_d)): the assembled
system against the oracle on a small mesh (explicit T_Omega region, a
spatially varying f, polynomial g) to the FP64 bars, the same L2 error from
both solutions, and the error falling with h over three GPU levels."""
import sys

import numpy as np
import pytest

import meshgen as mg
from meshgen import convergence as cv
import helpers as H

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


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


def _gpu_solve(dev, pb):
    import paper_2302_07499_amd as P
    _say(f"{pb.name} {pb.strategy} K={pb.mesh.n_tets} N={pb.mc_samples}")
    plan = dev.plan_problem(pb)
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    g = P.system_to_numpy(s)
    x, it, rr, ok = plan.solve(s, rtol=1e-12)
    assert ok, (it, rr)
    U = pb.g_nodal.copy()
    U[g["free_to_vertex"]] = x.cpu().numpy()
    plan.destroy()
    return g, U


def _oracle_solve(orc, pb):
    o = orc.problem_assemble(pb)
    x, it, rr, rc = orc.cg(o["ff_row_ptr"], o["ff_col"], o["ff_val"], o["rhs"], rtol=1e-12)
    U = pb.g_nodal.copy()
    U[o["free_to_vertex"]] = x
    return o, U


@pytest.mark.parametrize("strategy", ["fullcaps", "nocaps", "barycenter"])
def test_convergence_system_matches_oracle(dev, orc, strategy):
    pb = mg.convergence_problem(6, mc_samples=64, strategy=strategy)
    g, Ug = _gpu_solve(dev, pb)
    o, Uo = _oracle_solve(orc, pb)
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"  pairs {o['pair_counts']} errors {e}")
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL and e["rhs"] <= FP64_TOL, e
    sc = H.row_scale(o)
    for blk in ["ff", "fc"]:
        rows = np.repeat(np.arange(o["n_free"]), np.diff(o[blk + "_row_ptr"]))
        a, b = np.asarray(g[blk + "_val"]), np.asarray(o[blk + "_val"])
        big = np.abs(b) > 1e-4 * sc[rows]
        if big.any():
            assert np.max(np.abs(a - b)[big] / np.abs(b)[big]) <= FP64_TOL, blk
    # the two solutions and their errors
    assert np.max(np.abs(Ug - Uo)) <= 1e-9 * np.max(np.abs(Uo))
    eg = cv.l2_error(pb.mesh.coords, pb.mesh.tets, pb.tet_region, Ug)
    eo = cv.l2_error(pb.mesh.coords, pb.mesh.tets, pb.tet_region, Uo)
    _say(f"  L2 error gpu {eg:.6e} oracle {eo:.6e}")
    assert abs(eg - eo) <= 1e-6 * eo


def test_convergence_error_falls_with_h(dev):
    """fullcaps, N = 64: from h = 1/8 to h = 1/16 the L2 error falls at least
    like h^1.5 (measured about h^2 or faster)."""
    errs = []
    for m in (8, 12, 16):
        pb = mg.convergence_problem(m, mc_samples=64)
        g, U = _gpu_solve(dev, pb)
        errs.append(cv.l2_error(pb.mesh.coords, pb.mesh.tets, pb.tet_region, U))
        _say(f"  m={m} L2 error {errs[-1]:.4e}")
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] / errs[2] > 2.0 ** 1.5, errs
