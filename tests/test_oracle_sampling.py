"""Pins of the oracle's Monte Carlo sample test and sample keying.

* The sample test is the plain coordinate form of the fullcap definition
  (Sec. 4.2.2): y - p = sum_l lambda_l (X_l - p), accepted iff |y - p|^2 <
  delta^2 and y is not in U_I.  Its rounding band ("near ties") is checked
  against the same test evaluated in 80-bit extended precision: every sample
  whose double decision differs from the extended one must be reported as a
  near tie, and the oracle's |y - p|^2 must lie within the band of the
  extended value.  A sample placed exactly on the sphere is reported.
* Element keying (N samples per element E_m, reused by every outer point)
  draws the same points for every q and stays unbiased: the ball volume and
  the moments of every pair of a 6-tet cube agree with brute force.
"""
import math

import numpy as np
import pytest

import meshgen as mg

LD = np.longdouble


def _cut_pairs(orc, mesh, delta, count, rng):
    out = []
    K = mesh.n_tets
    while len(out) < count:
        n = int(rng.integers(K))
        k = int(rng.integers(4))
        p = orc.outer_point(mesh.coords, mesh.tets, n, k)
        cls = orc.classify_point(mesh.coords, mesh.tets, delta, p)
        cut = np.nonzero(cls >= orc.CLS_CUT0)[0]
        for m in rng.choice(cut, size=min(4, len(cut)), replace=False):
            out.append((n, k, int(m), p))
    return out


def _extended_decisions(orc, X, p, delta, N, seed, q, m, geo, keying):
    """|y - p|^2 and the acceptance of every sample in 80-bit arithmetic."""
    lam = np.array([orc.sample_lambda(seed, q, m, s, keying) for s in range(N)])
    e = X.astype(LD) - p.astype(LD)
    d = lam.astype(LD) @ e
    rr = (d * d).sum(axis=1)
    acc = rr < LD(delta) * LD(delta)
    if len(geo["planes"]):
        h = lam.astype(LD) @ geo["planes"].astype(LD).T
        acc &= ~np.all(h >= 0, axis=1)
    return rr, acc, e


@pytest.mark.parametrize("keying", ["pair", "element"])
def test_sample_test_band_covers_rounding(orc, keying):
    mesh = mg.kuhn_cube_mesh(5, jitter=0.2, seed=9)
    rng = np.random.default_rng(21)
    N = 512
    worst = 0.0
    total = 0
    flagged = 0
    for delta in [0.17, 0.31]:
        for (n, k, m, p) in _cut_pairs(orc, mesh, delta, 24, rng):
            q = 4 * n + k
            cls, rr, acc, tie = orc.pair_samples(mesh.coords, mesh.tets, n, k, m, delta, N, 5, keying=keying)
            geo = orc.pair_geometry(mesh.coords, mesh.tets, n, k, m, delta)
            X = mesh.coords[mesh.tets[m]]
            rr_x, acc_x, e = _extended_decisions(orc, X, p, delta, N, 5, q, m, geo, keying)
            E2 = float(np.max((e.astype(np.float64) ** 2).sum(axis=1)))
            band = 2.0 ** -40 * E2
            err = np.abs(rr.astype(LD) - rr_x).astype(np.float64)
            worst = max(worst, float(err.max() / band))
            # every decision that extended precision reverses is a reported near tie
            assert np.all(tie[acc != acc_x]), (n, k, m)
            total += N
            flagged += int(tie.sum())
    # the oracle's own rounding sits far inside the band, and near ties are rare
    print(f"worst oracle error / band = {worst:.3g}, near ties {flagged} of {total}")
    assert worst < 1.0 / 64, worst
    assert flagged <= 1e-4 * total, (flagged, total)


def test_sample_on_the_sphere_is_a_near_tie(orc):
    """Put the sphere through one sample: delta^2 = that sample's |y - p|^2
    (extended precision, rounded).  The oracle must report the sample."""
    mesh = mg.kuhn_cube_mesh(4, jitter=0.1, seed=3)
    rng = np.random.default_rng(2)
    delta0 = 0.3
    n, k, m, p = _cut_pairs(orc, mesh, delta0, 1, rng)[0]
    q = 4 * n + k
    N = 64
    X = mesh.coords[mesh.tets[m]]
    lam = np.array([orc.sample_lambda(7, q, m, s) for s in range(N)])
    e = X.astype(LD) - p.astype(LD)
    rr_x = ((lam.astype(LD) @ e) ** 2).sum(axis=1)
    hit = 0
    for s in range(N):
        delta = float(np.sqrt(rr_x[s]))
        cls, rr, acc, tie = orc.pair_samples(mesh.coords, mesh.tets, n, k, m, delta, N, 7)
        if cls < orc.CLS_CUT0:
            continue
        geo = orc.pair_geometry(mesh.coords, mesh.tets, n, k, m, delta)
        inU = len(geo["planes"]) and np.all(lam[s] @ geo["planes"].T >= 1e-9)
        if inU:
            continue  # the U_I test decides this sample, not the sphere
        assert tie[s], s
        hit += 1
    assert hit >= 10


def test_element_keying_reuses_samples_per_element(orc):
    for s in [0, 1, 7, 30]:
        a = orc.sample_lambda(11, 5, 9, s, "element")
        b = orc.sample_lambda(11, 123, 9, s, "element")
        c = orc.sample_lambda(11, 5, 10, s, "element")
        d = orc.sample_lambda(11, 5, 9, s, "pair")
        e = orc.sample_lambda(11, 123, 9, s, "pair")
        assert np.array_equal(a, b)
        assert not np.array_equal(a, c)
        assert not np.array_equal(d, e)
        assert not np.array_equal(a, d)
        assert a.sum() == 1.0 and np.all(a * 2 ** 21 == np.round(a * 2 ** 21))


def _brute_mc(X, p, delta, n, rng):
    lam = rng.dirichlet([1, 1, 1, 1], size=n)
    y = lam @ X
    acc = (np.sum((y - p) ** 2, axis=1) < delta * delta).astype(float)
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6
    f = np.concatenate([np.ones((n, 1)), lam,
                        np.stack([lam[:, i] * lam[:, j] for i in range(4) for j in range(i, 4)], 1)], 1)
    vals = vol * acc[:, None] * f
    return vals.mean(0), vals.std(0) / math.sqrt(n)


def test_element_keying_moments_vs_brute_force_mc(orc):
    """6-tet Kuhn cube, delta = 0.5: element-keyed fullcaps moments agree with
    a plain numpy Monte Carlo of E_m n B_delta(p) (z <= 5.5)."""
    mesh = mg.six_tet_cube_mesh()
    rng = np.random.default_rng(50)
    N, delta = 1 << 15, 0.5
    zmax = 0.0
    for n in range(6):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            for m in range(6):
                cls, S = orc.pair_moments(mesh.coords, mesh.tets, n, k, m, delta, N, 17, keying="element")
                if cls == orc.CLS_OUT:
                    continue
                X = mesh.coords[mesh.tets[m]]
                ref, se_ref = _brute_mc(X, p, delta, 200000, rng)
                vol = abs(np.linalg.det(X[1:] - X[0])) / 6
                se = np.sqrt(se_ref ** 2 + (vol * 0.5 / math.sqrt(N)) ** 2) + 1e-15
                zmax = max(zmax, float((np.abs(S - ref) / se).max()))
    assert zmax < 5.5, zmax


def test_element_keying_ball_volume_unbiased(orc):
    mesh = mg.kuhn_cube_mesh(10, jitter=0.2, seed=4)
    delta = 0.25
    exact = 4 / 3 * math.pi * delta ** 3
    pts = []
    for n in range(mesh.n_tets):
        p = orc.outer_point(mesh.coords, mesh.tets, n, 1)
        if np.all(p > delta + 1e-9) and np.all(p < 1 - delta - 1e-9):
            pts.append(n)
    rng = np.random.default_rng(8)
    for n in rng.choice(pts, size=2, replace=False):
        vals = [orc.point_moments(mesh.coords, mesh.tets, int(n), 1, delta, 64, seed, keying="element")[1][:, 0].sum()
                for seed in range(6)]
        v = np.array(vals)
        mean, se = v.mean(), v.std(ddof=1) / math.sqrt(len(v))
        assert abs(mean - exact) < 5 * se + 1e-14, (mean, exact, se)


def test_assembly_reports_no_near_ties_on_plain(orc):
    """The plain workload's 7.4e6 samples: the near-tie report is zero (so the
    GPU parity tests there compare at full precision)."""
    pb = mg.plain_problem()
    S = orc.problem_assemble(pb)
    assert S["near_ties"] == 0
    assert np.all(S["tie_allow"] == 0.0)
