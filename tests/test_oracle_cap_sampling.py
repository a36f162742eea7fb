"""Pins of cap sampling on E_m minus U_I (the corner tet for n_in = 3, three
cone tets from the first outside vertex for n_in = 1, 2): the region is
exactly E minus U_I, and sampling it estimates the same integrals as
sampling the whole element, with less variance.

* brute force: uniform points of E lie in exactly one sub-tet of the region
  when they are outside U_I (the half-space form of the fullcaps
  construction) and in none when inside; the region's volume plus that of
  U_I's subdivision is |E|;
* the approximate ball volume sum_m S0 at interior points is an unbiased
  estimate of |B_delta| = 4/3 pi delta^3 in both modes (mean over seeds within
  5 standard errors);
* per class n_in = 1, 2, 3, over all pairs of one point, the two modes agree
  in the mean of every moment summed over the pairs (within 5 standard errors
  of the difference), and that sum's S0 has a lower variance on E minus U_I
  (below 0.85 of the whole-element one, below half for n_in = 3);
* CUT(0) pairs are unchanged bit for bit; fewer than 3 samples are rejected.
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


def _tet_volume(X):
    return abs(np.linalg.det(X[1:] - X[0])) / 6.0


def test_region_tiles_e_minus_ui(orc, setup):
    mesh, delta, pts = setup
    rng = np.random.default_rng(7)
    seen = {1: 0, 2: 0, 3: 0}
    for (n, k, p) in pts:
        cls = orc.classify_point(mesh.coords, mesh.tets, delta, p)
        for code in (3, 4, 5):
            for m in np.nonzero(cls == code)[0][:6]:
                m = int(m)
                geo = orc.pair_geometry(mesh.coords, mesh.tets, n, k, m, delta)
                rows, vol = orc.cap_region(mesh.coords, mesh.tets, n, k, m, delta)
                nin = code - 2
                assert geo["n_in"] == nin and len(rows) == (1 if nin == 3 else 3)
                volE = _tet_volume(mesh.coords[mesh.tets[m]])
                # the region's volume and U_I's add up to |E|
                assert abs(vol.sum() + geo["subvol"].sum() - volE) <= 1e-12 * volE
                # its apex is an outside vertex (the same for every sub-tet)
                apex = rows[:, 0, :]
                assert np.all(apex == apex[0]) and np.count_nonzero(apex[0]) == 1
                o = int(np.argmax(apex[0]))
                r2 = np.sum((mesh.coords[mesh.tets[m]][o] - p) ** 2)
                assert r2 >= delta * delta
                # uniform points of E: in exactly one sub-tet iff outside U_I
                lam = rng.dirichlet(np.ones(4), size=3000)
                hp = lam @ geo["planes"].T                       # plane values
                inU = np.all(hp >= 0.0, axis=1)
                mu = np.stack([np.linalg.solve(rows[j].T, lam.T).T for j in range(len(rows))], axis=1)
                inT = np.all(mu >= 0.0, axis=2)                  # [points, sub-tets]
                clear = (np.min(np.abs(hp), axis=1) > 1e-9) & (np.min(np.abs(mu), axis=(1, 2)) > 1e-9)
                assert clear.sum() > 2500
                cnt = inT[clear].sum(axis=1)
                assert np.array_equal(cnt, np.where(inU[clear], 0, 1))
                seen[nin] += 1
    assert min(seen.values()) >= 6, seen


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


@pytest.fixture(scope="module")
def point_totals(orc, setup):
    """per seed, the moments of every pair of one interior point in both modes"""
    mesh, delta, pts = setup
    n, k, p = pts[2]
    out = {}
    for mode in ["whole", "outside_ui"]:
        runs = [orc.point_moments(mesh.coords, mesh.tets, n, k, delta, 16, s, cap_sampling=mode) for s in range(60)]
        out[mode] = np.array([S for _, S in runs])      # [seed, tet, 15]
        cls = runs[0][0]
    return cls, out


@pytest.mark.parametrize("code,max_ratio", [(5, 0.5), (4, 0.85), (3, 0.85)])
def test_region_sampling_same_mean_lower_variance(point_totals, code, max_ratio):
    """over all pairs of one class at one point: the moments summed over the
    pairs have the same mean in both modes, and their sum S0 a lower variance
    on E minus U_I"""
    cls, out = point_totals
    sel = cls == code
    assert sel.sum() >= 50
    totA = out["whole"][:, sel, :].sum(axis=1)
    totB = out["outside_ui"][:, sel, :].sum(axis=1)
    ns = totA.shape[0]
    se = np.sqrt(totA.var(axis=0, ddof=1) / ns + totB.var(axis=0, ddof=1) / ns)
    assert np.all(np.abs(totA.mean(axis=0) - totB.mean(axis=0)) <= 5 * se), (totA.mean(0) - totB.mean(0)) / se
    ratio = totB[:, 0].var(ddof=1) / totA[:, 0].var(ddof=1)
    assert ratio < max_ratio, ratio


def test_cut0_unchanged_and_few_samples_rejected(orc, setup):
    mesh, delta, pts = setup
    n, k, p = pts[2]
    cls = orc.classify_point(mesh.coords, mesh.tets, delta, p)
    c0 = np.nonzero(cls == 2)[0][:12]
    assert len(c0) >= 1
    for m in c0:
        a = orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, 3)[1]
        b = orc.pair_moments(mesh.coords, mesh.tets, n, k, int(m), delta, 16, 3, cap_sampling="outside_ui")[1]
        assert np.array_equal(a, b)
    vf = mg.free_mask_box(mesh.coords, delta)
    with pytest.raises(RuntimeError):
        orc.assemble(mesh.coords, mesh.tets, vf, delta, 1.0, 2, 0, cap_sampling="outside_ui")
