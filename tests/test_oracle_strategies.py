"""Pins of the oracle's ball approximation strategies (Sec. 4.1: barycenter,
overlap, inside, nocaps beside fullcaps), checked without the oracle's own
arithmetic where possible:

* inside / barycenter: the approximate-ball volume sum_m S0 equals the volume
  of the tets selected by an independent numpy test (all vertices in the open
  ball; barycenter in the open ball);
* overlap: the selected tets are those the (separately pinned) classifier finds
  meeting the ball, and their union covers the ball: |B| <= volume <= |B_(delta+h)|;
* nocaps: volume = inside tets + the closed-form-pinned T_I volumes, and the
  polytope is inscribed, between |B_(delta - h^2/(4 delta))| and |B_delta|
  (Lemma nocaps);
* all: B_(delta-h) within B_(delta,h) within B_(delta+h) in volume (the bound
  of the approximation theorem), and the assembled system keeps symmetry and
  A_full 1 = 0.
"""
import math

import numpy as np
import pytest

import meshgen as mg

STRATS = ["nocaps", "overlap", "inside", "barycenter"]


@pytest.fixture(scope="module")
def setup(orc):
    mesh = mg.kuhn_cube_mesh(10, jitter=0.2, seed=4)
    delta = 0.25
    X = mesh.coords[mesh.tets]
    vol = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    h = max(np.linalg.norm(X[:, a] - X[:, b], axis=1).max() for a, b in edges)
    pts = []
    for n in range(0, mesh.n_tets, 7):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            if np.all(p > delta + 1e-9) and np.all(p < 1 - delta - 1e-9):
                pts.append((n, k, p))
    rng = np.random.default_rng(1)
    sel = rng.choice(len(pts), size=4, replace=False)
    return mesh, X, vol, h, delta, [pts[i] for i in sel]


def _ballvol(r):
    return 4 / 3 * math.pi * max(r, 0.0) ** 3


@pytest.mark.parametrize("strategy", STRATS)
def test_strategy_volume_and_selection(orc, setup, strategy):
    mesh, X, vol, h, delta, pts = setup
    d2 = delta * delta
    for (n, k, p) in pts:
        cls, S = orc.point_moments(mesh.coords, mesh.tets, n, k, delta, 16, 0, strategy=strategy)
        V = S[:, 0].sum()
        r2 = ((X - p) ** 2).sum(axis=2)
        if strategy == "inside":
            sel = np.all(r2 < d2, axis=1)
            assert np.array_equal(cls != 0, sel)
            assert abs(V - vol[sel].sum()) <= 1e-12 * V
        elif strategy == "barycenter":
            c = X.mean(axis=1)
            sel = ((c - p) ** 2).sum(axis=1) < d2
            assert np.array_equal(cls != 0, sel)
            assert abs(V - vol[sel].sum()) <= 1e-12 * V
        elif strategy == "overlap":
            full = orc.classify_point(mesh.coords, mesh.tets, delta, p)
            assert np.array_equal(cls != 0, full != 0)
            assert np.all(cls[cls != 0] == 1)
            assert _ballvol(delta) <= V <= _ballvol(delta + h)
        else:  # nocaps
            full = orc.classify_point(mesh.coords, mesh.tets, delta, p)
            V_in = vol[full == 1].sum()
            V_ti = 0.0
            for m in np.nonzero(full >= 3)[0]:
                g = orc.pair_geometry(mesh.coords, mesh.tets, n, k, int(m), delta)
                V_ti += g["subvol"].sum()
            assert np.all((cls != 0) == (full == 1) | (full >= 3))
            assert abs(V - (V_in + V_ti)) <= 1e-12 * V
            assert _ballvol(delta - h * h / (4 * delta)) - 1e-12 <= V <= _ballvol(delta)
        assert _ballvol(delta - h) <= V <= _ballvol(delta + h)
        # every selected pair is integrated whole (4-point rule) except nocaps' cut tets
        if strategy != "nocaps":
            ss = cls != 0
            assert np.allclose(S[ss, 0], vol[ss], rtol=1e-13, atol=0)


@pytest.mark.parametrize("strategy", STRATS)
def test_strategy_system_symmetry_and_rowsums(orc, strategy):
    pb = mg.plain_problem()
    pb.strategy = strategy
    S = orc.problem_assemble(pb)
    nf = S["n_free"]
    A = np.zeros((nf, pb.mesh.n_vertices))
    f2v = S["free_to_vertex"]
    for r in range(nf):
        for e in range(S["ff_row_ptr"][r], S["ff_row_ptr"][r + 1]):
            A[r, f2v[S["ff_col"][e]]] += S["ff_val"][e]
        for e in range(S["fc_row_ptr"][r], S["fc_row_ptr"][r + 1]):
            A[r, S["fc_col"][e]] += S["fc_val"][e]
    Aff = A[:, f2v]
    scale = np.abs(A).sum(1)
    assert np.max(np.abs(Aff - Aff.T)) <= 1e-14 * scale.max()
    assert np.all(np.abs(A.sum(1)) <= 1e-12 * scale)
    # only fullcaps samples: the other strategies are deterministic in the seed
    pb2 = mg.plain_problem()
    pb2.strategy = strategy
    pb2.seed = 7
    S2 = orc.problem_assemble(pb2)
    assert np.array_equal(S["ff_val"], S2["ff_val"]) and np.array_equal(S["rhs"], S2["rhs"])
