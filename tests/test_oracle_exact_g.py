"""Pins of the oracle's paper-exact right-hand side (eq. F1.5 with F_h of
eq. Fh: g itself inside the inner integrals over Omega_I), which it sums term
by term in the paper's form, against the nodal-constraint form and closed
forms:

* g linear: its nodal interpolant is exact, so both right-hand sides agree;
* delta beyond the mesh, g quadratic: every pair is IN and the 4-point rule is
  exact for g, so the difference is 2 psi D m_i with D = int over Omega_I of
  (g - g_h) (closed-form tet integrals) and m_i = int over T_Omega of phi_i;
* the matrix blocks do not depend on the right-hand side form.
"""
import numpy as np
import pytest

import meshgen as mg
from meshgen import convergence as cv


def _lin_poly():
    G = np.zeros((2, 2, 2))
    G[0, 0, 0], G[1, 0, 0], G[0, 1, 0], G[0, 0, 1] = 0.3, 0.5, -0.2, 0.7
    return G, lambda x: 0.3 + 0.5 * x[..., 0] - 0.2 * x[..., 1] + 0.7 * x[..., 2]


def _scale(S):
    return max(1e-300, float(np.max(np.abs(S["rhs"]))))


@pytest.mark.parametrize("strategy", ["fullcaps", "nocaps", "overlap"])
def test_linear_g_gives_the_nodal_rhs(orc, strategy):
    pb = mg.convergence_problem(4, mc_samples=16, strategy=strategy)
    G, g = _lin_poly()
    pb.g_nodal = g(pb.mesh.coords)
    pb.g_poly = G
    a = orc.problem_assemble(pb)
    b = orc.problem_assemble(pb, exact_g=True)
    for k in ["ff_val", "fc_val", "ff_col", "fc_col"]:
        assert np.array_equal(a[k], b[k]), k
    assert np.max(np.abs(a["rhs"] - b["rhs"])) <= 1e-13 * _scale(a)


def _quad_int(X, Q):
    """int over the tet X [4,3] of y^T Q y + (closed form for quadratics):
    int y_i y_j = |T|/20 (sum_a X_ai X_aj + s_i s_j), s = sum_a X_a."""
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6.0
    s = X.sum(axis=0)
    M = vol / 20.0 * (X.T @ X + np.outer(s, s))
    return float(np.sum(Q * M)), vol


def test_large_horizon_quadratic_g_closed_form(orc):
    mesh = mg.kuhn_cube_mesh(3, jitter=0.1, seed=4)
    V, K = mesh.n_vertices, mesh.n_tets
    vfree = mg.free_mask_box(mesh.coords, 0.2)
    assert 0 < vfree.sum() < V
    delta, psi = 10.0, 0.9
    Q = np.array([[1.0, 0.2, 0.0], [0.2, -0.5, 0.3], [0.0, 0.3, 0.8]])
    g = lambda x: np.einsum("...i,ij,...j->...", x, Q, x)
    G = np.zeros((3, 3, 3))
    G[2, 0, 0], G[0, 2, 0], G[0, 0, 2] = Q[0, 0], Q[1, 1], Q[2, 2]
    G[1, 1, 0], G[1, 0, 1], G[0, 1, 1] = 2 * Q[0, 1], 2 * Q[0, 2], 2 * Q[1, 2]
    gn = g(mesh.coords)
    a = orc.assemble(mesh.coords, mesh.tets, vfree, delta, psi, 8, 0, g_nodal=gn)
    b = orc.assemble(mesh.coords, mesh.tets, vfree, delta, psi, 8, 0, g_nodal=gn, g_poly=G)
    assert a["pair_counts"][1:].sum() == 0
    region = vfree[mesh.tets].any(axis=1)
    D = 0.0
    mO = np.zeros(V)
    for e, t in enumerate(mesh.tets):
        X = mesh.coords[t]
        gi, vol = _quad_int(X, Q)
        if region[e]:
            mO[t] += vol / 4.0
        else:
            D += gi - vol / 4.0 * gn[t].sum()
    expect = 2.0 * psi * D * mO[a["free_to_vertex"]]
    diff = b["rhs"] - a["rhs"]
    assert abs(D) > 1e-4
    assert np.max(np.abs(diff - expect)) <= 1e-12 * max(_scale(a), np.max(np.abs(expect)))


def test_exact_g_changes_the_rhs_only_by_the_defect(orc):
    """u as g on the convergence mesh: the two right-hand sides differ (u is
    not affine), by much less than the rhs itself, and the matrices agree."""
    pb = mg.convergence_problem(4, mc_samples=16)
    a = orc.problem_assemble(pb)
    b = orc.problem_assemble(pb, exact_g=True)
    assert np.array_equal(a["ff_val"], b["ff_val"]) and np.array_equal(a["fc_val"], b["fc_val"])
    d = np.max(np.abs(a["rhs"] - b["rhs"]))
    assert 0.0 < d < 0.1 * _scale(a)


def test_exact_g_rejects_corner_sampling(orc):
    pb = mg.convergence_problem(3, mc_samples=8)
    pb.cap_sampling = "outside_ui"
    with pytest.raises(RuntimeError):
        orc.problem_assemble(pb, exact_g=True)
