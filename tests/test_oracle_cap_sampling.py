"""Pins of cap sampling on E_m minus U_I (the corner tet for n_in = 3): it
estimates the same integrals as sampling the whole element, with less
variance.

* the approximate ball volume sum_m S0 at interior points is an unbiased
  estimate of |B_delta| = 4/3 pi delta^3 in both modes (mean over seeds within
  5 standard errors);
* on n_in = 3 pairs the two modes agree in the mean of every moment summed
  over the pairs (within 5 standard errors of the difference), and the median
  per-pair variance of S0 in the corner mode is below half the whole-element
  one;
* pairs with n_in != 3 are unchanged bit for bit.
"""
import math

import numpy as np
import pytest

import meshgen as mg


@pytest.fixture(scope="module")
def setup(orc):
    mesh = mg.kuhn_cube_mesh(10, jitter=0.2, seed=4)
    delta = 0.25
    pts = []
    for n in range(0, mesh.n_tets, 5):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            if np.all(p > delta + 1e-9) and np.all(p < 1 - delta - 1e-9):
                pts.append((n, k, p))
    rng = np.random.default_rng(2)
    sel = rng.choice(len(pts), size=3, replace=False)
    return mesh, delta, [pts[i] for i in sel]


def test_ball_volume_unbiased_both_modes(orc, setup):
    mesh, delta, pts = setup
    exact = 4 / 3 * math.pi * delta ** 3
    for (n, k, p) in pts[:2]:
        for mode in ["whole", "outside_ui"]:
            vals = [orc.point_moments(mesh.coords, mesh.tets, n, k, delta, 32, seed, cap_sampling=mode)[1][:, 0].sum()
                    for seed in range(8)]
            v = np.array(vals)
            se = v.std(ddof=1) / math.sqrt(len(v))
            assert abs(v.mean() - exact) < 5 * se + 1e-14, (mode, v.mean(), exact, se)


def test_corner_sampling_same_mean_lower_variance(orc, setup):
    mesh, delta, pts = setup
    n, k, p = pts[2]
    cls = orc.classify_point(mesh.coords, mesh.tets, delta, p)
    c3 = np.nonzero(cls == 5)[0][:12]       # CUT with 3 inside vertices
    other = np.nonzero((cls >= 2) & (cls != 5))[0][:12]
    assert len(c3) >= 6 and len(other) >= 6
    seeds = range(60)
    ratios = []
    totA = np.zeros((len(seeds), 15))
    totB = np.zeros((len(seeds), 15))
    for m in c3:
        A = np.array([orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, s)[1] for s in seeds])
        B = np.array([orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, s,
                                       cap_sampling="outside_ui")[1] for s in seeds])
        totA += A
        totB += B
        ratios.append(B[:, 0].var(ddof=1) / max(A[:, 0].var(ddof=1), 1e-300))
    # the moments summed over the pairs: same mean in both modes
    se = np.sqrt(totA.var(axis=0, ddof=1) / len(seeds) + totB.var(axis=0, ddof=1) / len(seeds))
    assert np.all(np.abs(totA.mean(axis=0) - totB.mean(axis=0)) <= 5 * se), (totA.mean(0) - totB.mean(0)) / se
    assert np.median(ratios) < 0.5, ratios
    for m in other:
        a = orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, 3)[1]
        b = orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, 3, cap_sampling="outside_ui")[1]
        assert np.array_equal(a, b)
