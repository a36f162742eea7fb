"""Paper-exact right-hand side on the GPU (nlfem_assemble_exact_g: g itself
inside the inner integrals over Omega_I, eqs. Fh and F1.5) against the
oracle's term-by-term form: the right-hand side within 1e-12 of its scale,
the matrix blocks bitwise those of nlfem_assemble; a linear g reproduces the
nodal right-hand side; bad arguments are rejected at the boundary."""
import sys

import numpy as np
import pytest

import meshgen as mg
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


def _both(dev, pb):
    import paper_2302_07499_amd as P
    _say(f"{pb.name} {pb.strategy} K={pb.mesh.n_tets} N={pb.mc_samples}")
    plan = dev.plan_problem(pb)
    a = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal))
    b = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal, g_poly=pb.g_poly))
    plan.destroy()
    return a, b


@pytest.mark.parametrize("strategy", ["fullcaps", "nocaps", "overlap"])
def test_exact_g_matches_oracle(dev, orc, strategy):
    pb = mg.convergence_problem(6, mc_samples=64, strategy=strategy)
    a, b = _both(dev, pb)
    for k in ["ff_val", "fc_val", "ff_col", "fc_col", "ff_row_ptr", "fc_row_ptr"]:
        assert np.array_equal(a[k], b[k]), k
    o = orc.problem_assemble(pb, exact_g=True)
    H.pattern_equal(b, o)
    scale = float(np.max(np.abs(o["rhs"])))
    err = float(np.max(np.abs(b["rhs"] - o["rhs"]))) / scale
    moved = float(np.max(np.abs(b["rhs"] - a["rhs"]))) / scale
    _say(f"  rhs error vs oracle {err:.3e} (exact-g minus nodal rhs: {moved:.3e} of the scale)")
    assert err <= FP64_TOL
    assert moved > 1e3 * FP64_TOL


def test_linear_g_reproduces_nodal_rhs(dev):
    pb = mg.convergence_problem(5, mc_samples=32)
    G = np.zeros((2, 2, 2))
    G[0, 0, 0], G[1, 0, 0], G[0, 1, 0], G[0, 0, 1] = 0.3, 0.5, -0.2, 0.7
    x = pb.mesh.coords
    pb.g_nodal = 0.3 + 0.5 * x[:, 0] - 0.2 * x[:, 1] + 0.7 * x[:, 2]
    pb.g_poly = G
    a, b = _both(dev, pb)
    d = float(np.max(np.abs(a["rhs"] - b["rhs"]))) / float(np.max(np.abs(a["rhs"])))
    _say(f"  linear g: |rhs_exact - rhs_nodal| / scale = {d:.3e}")
    assert d <= 1e-13


def test_exact_g_argument_errors(dev):
    import paper_2302_07499_amd as P
    pb = mg.convergence_problem(3, mc_samples=8)
    plan = dev.plan_problem(pb)
    with pytest.raises(P.NlfemError):
        plan.assemble(pb.f_qp, pb.g_nodal, g_poly=np.zeros((6, 6, 6)))  # degree 5 > 4
    plan.destroy()
    pb.cap_sampling = "outside_ui"
    plan = dev.plan_problem(pb)
    with pytest.raises(P.NlfemError):
        plan.assemble(pb.f_qp, pb.g_nodal, g_poly=pb.g_poly)
    plan.destroy()
