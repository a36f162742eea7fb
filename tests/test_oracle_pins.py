"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: textbook
identities, published known-answer vectors, closed forms, an independent
library routine (scipy's Qhull hull volume and SLSQP distance), brute-force
Monte Carlo with numpy's own generator, or invariants of the bilinear form.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial import ConvexHull

import meshgen as mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- quadrature --
def test_rule_constants_and_mass_identity(orc):
    """4-point degree-2 rule (Sec. 4.2.1): weights 1/4; sum_r K_r/4 = 1/4 and
    sum_r K_r K_r^T / 4 = (1 + delta_ij)/20 (P1 mass matrix on the reference tet)."""
    a, b = orc.rule_constants()
    assert a == (5 + 3 * math.sqrt(5)) / 20 and b == (5 - math.sqrt(5)) / 20
    K = np.full((4, 4), b) + np.eye(4) * (a - b)
    assert np.allclose(K.sum(0) / 4, 0.25, rtol=0, atol=1e-16)
    M = (K.T @ K) / 4
    assert np.allclose(M, (np.ones((4, 4)) + np.eye(4)) / 20, rtol=0, atol=1e-16)


def test_outer_points_integrate_quadratics(orc):
    """Outer points p_k with weights |E|/4 integrate x_i x_j exactly on a tet
    (degree-2 exactness), against the closed form |E|/20 (sum_a X_a X_a^T + S S^T)."""
    rng = np.random.default_rng(0)
    X = rng.normal(size=(4, 3))
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6
    P = np.array([orc.outer_point(X, tets, 0, k) for k in range(4)])
    quad = (vol / 4) * P.T @ P
    S = X.sum(0)
    exact = vol / 20 * (X.T @ X + np.outer(S, S))
    assert np.allclose(quad, exact, rtol=1e-13, atol=1e-14)
    assert np.allclose(P.mean(0), X.mean(0), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------- RNG --
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_tet_sampling_is_uniform_dirichlet(orc):
    """Barycentric samples: exact multiples of 2^-21 summing to exactly 1, and
    uniform on the simplex: E[l_i] = 1/4, E[l_i l_j] = (1 + delta_ij)/20,
    marginal l_0 ~ Beta(1, 3) (KS distance)."""
    n = 40000
    L = np.array([orc.sample_lambda(12345, 7, 11, s) for s in range(n)])
    assert np.all(L.sum(1) == 1.0)
    assert np.all(L * 2 ** 21 == np.round(L * 2 ** 21))
    assert np.all(L >= 0)
    se = 0.5 / math.sqrt(n)
    assert np.all(np.abs(L.mean(0) - 0.25) < 5 * se)
    M = L.T @ L / n
    assert np.all(np.abs(M - (np.ones((4, 4)) + np.eye(4)) / 20) < 5 * 0.3 / math.sqrt(n))
    x = np.sort(L[:, 0])
    cdf = 1 - (1 - x) ** 3
    ks = np.max(np.abs(cdf - np.arange(1, n + 1) / n))
    assert ks < 1.63 / math.sqrt(n) * 1.2
    # the even and odd halves of one Philox call are not correlated
    c = np.corrcoef(L[0::2, 0], L[1::2, 0])[0, 1]
    assert abs(c) < 5 / math.sqrt(n / 2)


# ---------------------------------------------------------- classification --
def _tet():
    return np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]]), np.array([[0, 1, 2, 3]],
                                                                                     dtype=np.int32)


def test_classification_hand_cases(orc):
    """Def. of the dividing strategy: open ball, vertex counts, and the
    all-vertices-outside-but-intersecting case."""
    X, T = _tet()
    c = lambda d, p: int(orc.classify_point(X, T, d, np.array(p, dtype=float))[0])
    assert c(0.5, [5.0, 5.0, 5.0]) == orc.CLS_OUT
    assert c(2.0, [0.25, 0.25, 0.25]) == orc.CLS_IN
    assert c(0.5, [0.0, 0.0, 0.0]) == orc.CLS_CUT0 + 1          # only the origin vertex inside
    assert c(0.75, [0.5, 0.0, 0.0]) == orc.CLS_CUT0 + 2         # vertices 0 and 1
    assert c(0.9, [0.4, 0.4, 0.0]) == orc.CLS_CUT0 + 3          # vertices 0,1,2
    assert c(0.1, [0.2, 0.2, 0.2]) == orc.CLS_CUT0              # ball strictly inside the tet
    assert c(0.25, [0.25, 0.25, -0.125]) == orc.CLS_CUT0        # ball pokes through face z=0
    assert c(0.125, [0.25, 0.25, -0.125]) == orc.CLS_OUT        # touches face z=0: open ball -> OUT
    assert c(1.0, [2.0, 0.0, 0.0]) == orc.CLS_OUT               # vertex at distance exactly delta
    assert c(0.25, [0.5, -0.125, -0.125]) == orc.CLS_CUT0       # near the edge x-axis only


def _dist_point_tet(X, p):
    """Independent distance from p to a tet: minimise |sum lam_l X_l - p| over the simplex (SLSQP)."""
    f = lambda l: float(np.sum((l @ X - p) ** 2))
    cons = [{"type": "eq", "fun": lambda l: l.sum() - 1.0}]
    best = np.inf
    for start in np.vstack([np.full(4, 0.25), np.eye(4)]):
        r = minimize(f, start, bounds=[(0, 1)] * 4, constraints=cons, method="SLSQP",
                     options={"ftol": 1e-15, "maxiter": 400})
        best = min(best, r.fun)
    return math.sqrt(max(best, 0.0))


def test_classification_matches_independent_distance(orc):
    """Random tets/points: non-OUT iff dist(p, tet) < delta (checked away from ties)."""
    rng = np.random.default_rng(1)
    T = np.array([[0, 1, 2, 3]], dtype=np.int32)
    checked = 0
    for _ in range(300):
        X = rng.normal(size=(4, 3))
        p = rng.normal(size=3) * 1.5
        delta = rng.uniform(0.2, 1.5)
        d = _dist_point_tet(X, p)
        if abs(d - delta) < 1e-4:
            continue
        cls = int(orc.classify_point(X, T, delta, p)[0])
        assert (cls != orc.CLS_OUT) == (d < delta)
        nin = int(np.sum(np.sum((X - p) ** 2, 1) < delta * delta))
        if cls != orc.CLS_OUT:
            assert cls == (orc.CLS_IN if nin == 4 else orc.CLS_CUT0 + nin)
        checked += 1
    assert checked > 250


# ------------------------------------------------------------- cut geometry --
def _cut_pairs(orc, mesh, delta, want, limit=40):
    """(n, k, m) pairs of a mesh with class CUT(n_in) for n_in in want."""
    out = []
    for n in range(0, mesh.n_tets, 7):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            cls = orc.classify_point(mesh.coords, mesh.tets, delta, p)
            for m in np.nonzero(cls >= orc.CLS_CUT0)[0]:
                nin = int(cls[m]) - orc.CLS_CUT0
                if nin in want:
                    out.append((n, k, int(m), nin, p))
            if len(out) >= limit:
                return out
    return out


@pytest.fixture(scope="module")
def jmesh():
    return mg.kuhn_cube_mesh(5, jitter=0.2, seed=3)


def test_edge_points_lie_on_sphere(orc, jmesh):
    delta = 0.37
    pairs = _cut_pairs(orc, jmesh, delta, {1, 2, 3}, limit=120)
    assert len(pairs) > 50
    for (n, k, m, nin, p) in pairs:
        g = orc.pair_geometry(jmesh.coords, jmesh.tets, n, k, m, delta)
        X = jmesh.coords[jmesh.tets[m]]
        r = np.linalg.norm(X - p, axis=1)
        I = np.nonzero(r < delta)[0]
        O = np.nonzero(r >= delta)[0]
        assert g["n_in"] == len(I) == nin
        for a in I:
            for b in O:
                t = g["t"][a, b]
                assert 0 < t <= 1
                y = X[a] + t * (X[b] - X[a])
                assert abs(np.linalg.norm(y - p) - delta) < 1e-13


def test_subdivision_volumes_closed_forms_and_hull(orc, jmesh):
    """T_I volumes: n_in=1 -> |E| t_ab t_ac t_ad; n_in=3 -> |E| (1 - prod(1 - t_xd));
    n_in=2 -> volume of conv(I u P) by Qhull.  Also: U_I's vertices are in the
    closed ball and satisfy every half-space of the chosen split."""
    delta = 0.41
    pairs = _cut_pairs(orc, jmesh, delta, {1, 2, 3}, limit=200)
    seen = set()
    for (n, k, m, nin, p) in pairs:
        g = orc.pair_geometry(jmesh.coords, jmesh.tets, n, k, m, delta)
        X = jmesh.coords[jmesh.tets[m]]
        vol = abs(np.linalg.det(X[1:] - X[0])) / 6
        r = np.linalg.norm(X - p, axis=1)
        I = list(np.nonzero(r < delta)[0]); O = list(np.nonzero(r >= delta)[0])
        t = g["t"]
        total = g["subvol"].sum()
        if nin == 1:
            a = I[0]
            exact = vol * t[a, O[0]] * t[a, O[1]] * t[a, O[2]]
        elif nin == 3:
            d = O[0]
            exact = vol * (1 - (1 - t[I[0], d]) * (1 - t[I[1], d]) * (1 - t[I[2], d]))
        else:
            pts = [X[a] for a in I]
            for a in I:
                for b in O:
                    pts.append(X[a] + t[a, b] * (X[b] - X[a]))
            exact = ConvexHull(np.array(pts)).volume
        assert abs(total - exact) <= 1e-11 * vol, (nin, total, exact)
        for s in range(g["sub"].shape[0]):
            for row in g["sub"][s]:
                y = row @ X
                assert np.linalg.norm(y - p) <= delta * (1 + 1e-12)
                for c in g["planes"]:
                    assert float(c @ row) >= -1e-12 * np.abs(c).sum()
        seen.add(nin)
    assert seen == {1, 2, 3}


def test_inscribed_faces_respect_lemma_nocaps(orc, jmesh):
    """Lemma (nocaps): points of a face whose vertices lie on the sphere with
    mutual distances <= h are farther than delta - h^2/(4 delta) from p."""
    delta = 0.37
    rng = np.random.default_rng(5)
    pairs = _cut_pairs(orc, jmesh, delta, {1, 3}, limit=60)
    for (n, k, m, nin, p) in pairs:
        g = orc.pair_geometry(jmesh.coords, jmesh.tets, n, k, m, delta)
        X = jmesh.coords[jmesh.tets[m]]
        r = np.linalg.norm(X - p, axis=1)
        I = list(np.nonzero(r < delta)[0]); O = list(np.nonzero(r >= delta)[0])
        t = g["t"]
        if nin == 1:
            F = [X[I[0]] + t[I[0], b] * (X[b] - X[I[0]]) for b in O]
        else:
            F = [X[a] + t[a, O[0]] * (X[O[0]] - X[a]) for a in I]
        F = np.array(F)
        h = max(np.linalg.norm(F[i] - F[j]) for i in range(3) for j in range(3))
        w = rng.dirichlet([1, 1, 1], size=200)
        y = w @ F
        assert np.all(np.linalg.norm(y - p, axis=1) > delta - h * h / (4 * delta) - 1e-14)


# -------------------------------------------------------- Monte Carlo caps --
def test_plane_cap_volume(orc):
    """A tet containing B_delta(p) except the cap cut off by one face plane at
    distance rho: E[S0] = 4/3 pi delta^3 - pi (delta - rho)^2 (2 delta + rho)/3."""
    delta, rho = 1.0, 0.4
    # face z = -rho; apex high above; base wide enough that the other faces are > delta away
    X = np.array([[-6.0, -6.0, -rho], [9.0, -6.0, -rho], [-6.0, 9.0, -rho], [-1.5, -1.5, 12.0]])
    T = np.array([[0, 1, 2, 3]], dtype=np.int32)
    p = np.zeros(3)
    assert int(orc.classify_point(X, T, delta, p)[0]) == orc.CLS_CUT0
    N = 400000
    # a small helper tet whose outer point k=0 sits at the origin
    a, b = orc.rule_constants()
    Y = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, -1, -1]], dtype=float) * 1e-3
    Y -= (a * Y[0] + b * (Y[1] + Y[2] + Y[3]))  # put outer point k=0 at the origin (up to rounding)
    allc = np.vstack([Y, X])
    allt = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], dtype=np.int32)
    q = orc.outer_point(allc, allt, 0, 0)
    assert np.all(np.abs(q) < 1e-15)
    cls, S = orc.pair_moments(allc, allt, 0, 0, 1, delta, N, 99)
    assert cls == orc.CLS_CUT0
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6
    exact = 4 / 3 * math.pi * delta ** 3 - math.pi * (delta - rho) ** 2 * (2 * delta + rho) / 3
    phat = exact / vol
    se = vol * math.sqrt(phat * (1 - phat) / N)
    assert abs(S[0] - exact) < 5 * se, (S[0], exact, se)


def _brute_mc(X, p, delta, n, rng):
    lam = rng.dirichlet([1, 1, 1, 1], size=n)
    y = lam @ X
    acc = (np.sum((y - p) ** 2, axis=1) < delta * delta).astype(float)
    vol = abs(np.linalg.det(X[1:] - X[0])) / 6
    f = np.concatenate([np.ones((n, 1)), lam,
                        np.stack([lam[:, i] * lam[:, j] for i in range(4) for j in range(i, 4)], 1)], 1)
    vals = vol * acc[:, None] * f
    return vals.mean(0), vals.std(0) / math.sqrt(n)


@pytest.mark.parametrize("delta", [0.3, 0.5, 0.8])
def test_fullcaps_moments_vs_brute_force_mc(orc, delta):
    """6-tet Kuhn cube: fullcaps moments (exact T_I + MC on the fullcap) agree with
    a plain numpy Monte Carlo of E_m n B_delta(p) with no subdivision (z <= 5)."""
    mesh = mg.six_tet_cube_mesh()
    rng = np.random.default_rng(int(delta * 100))
    N = 1 << 15
    zmax = 0.0
    for n in range(6):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            for m in range(6):
                cls, S = orc.pair_moments(mesh.coords, mesh.tets, n, k, m, delta, N, 7 + n)
                X = mesh.coords[mesh.tets[m]]
                if cls == orc.CLS_OUT:
                    continue
                ref, se_ref = _brute_mc(X, p, delta, 200000, rng)
                vol = abs(np.linalg.det(X[1:] - X[0])) / 6
                se = np.sqrt(se_ref ** 2 + (vol * 0.5 / math.sqrt(N)) ** 2) + 1e-15
                z = np.abs(S - ref) / se
                zmax = max(zmax, float(z.max()))
    assert zmax < 5.5, zmax


# --------------------------------------------------------- ball functionals --
@pytest.fixture(scope="module")
def interior_points(orc):
    mesh = mg.kuhn_cube_mesh(10, jitter=0.2, seed=4)
    delta = 0.25
    pts = []
    for n in range(mesh.n_tets):
        for k in range(4):
            p = orc.outer_point(mesh.coords, mesh.tets, n, k)
            if np.all(p > delta + 1e-9) and np.all(p < 1 - delta - 1e-9):
                pts.append((n, k, p))
    rng = np.random.default_rng(0)
    sel = rng.choice(len(pts), size=6, replace=False)
    return mesh, delta, [pts[i] for i in sel]


def _seeds_stats(vals):
    v = np.array(vals)
    return v.mean(), v.std(ddof=1) / math.sqrt(len(v))


def test_ball_volume_at_interior_points(orc, interior_points):
    """sum_m S0 is an unbiased estimate of |B_delta| = 4/3 pi delta^3 where the ball
    stays inside the mesh (fullcaps = exact T_I + unbiased MC over the caps)."""
    mesh, delta, pts = interior_points
    exact = 4 / 3 * math.pi * delta ** 3
    for (n, k, p) in pts[:3]:
        vals = []
        for seed in range(6):
            cls, S = orc.point_moments(mesh.coords, mesh.tets, n, k, delta, 64, seed)
            vals.append(S[:, 0].sum())
        mean, se = _seeds_stats(vals)
        assert abs(mean - exact) < 5 * se + 1e-14, (mean, exact, se)
        assert abs(mean - exact) / exact < 2e-3


def test_nonlocal_operator_on_x1_squared(orc, interior_points):
    """With psi = 15/(4 pi delta^5), L x1^2 = 2 psi int_B (y1^2 - p1^2) dy = 2 at
    interior points; from the moments, int y1^2 = sum_ab S2_ab X_a1 X_b1."""
    mesh, delta, pts = interior_points
    psi = mg.psi_unit_laplacian(delta)
    iu = [(i, j) for i in range(4) for j in range(i, 4)]
    for (n, k, p) in pts[3:]:
        vals = []
        for seed in range(6):
            cls, S = orc.point_moments(mesh.coords, mesh.tets, n, k, delta, 64, seed)
            tot = 0.0
            for m in np.nonzero(cls != 0)[0]:
                x = mesh.coords[mesh.tets[m], 0]
                s2 = 0.0
                for t_, (i, j) in enumerate(iu):
                    s2 += S[m, 5 + t_] * x[i] * x[j] * (1 if i == j else 2)
                tot += s2 - p[0] ** 2 * S[m, 0]
            vals.append(2 * psi * tot)
        mean, se = _seeds_stats(vals)
        assert abs(mean - 2.0) < 5 * se + 1e-12, (mean, se)


# ------------------------------------------------------------- assembled system --
def _dense(S, n_vertices):
    nf = S["n_free"]
    A = np.zeros((nf, n_vertices))
    f2v = S["free_to_vertex"]
    for r in range(nf):
        for e in range(S["ff_row_ptr"][r], S["ff_row_ptr"][r + 1]):
            A[r, f2v[S["ff_col"][e]]] += S["ff_val"][e]
        for e in range(S["fc_row_ptr"][r], S["fc_row_ptr"][r + 1]):
            A[r, S["fc_col"][e]] += S["fc_val"][e]
    return A


@pytest.fixture(scope="module")
def plain_sys(orc):
    pb = mg.plain_problem()
    return pb, orc.problem_assemble(pb)


def test_plain_symmetry_rowsums_spd(orc, plain_sys):
    pb, S = plain_sys
    A = _dense(S, pb.mesh.n_vertices)
    f2v = S["free_to_vertex"]
    Aff = A[:, f2v]
    scale = np.abs(A).sum(1)
    assert np.max(np.abs(Aff - Aff.T)) <= 1e-14 * scale.max()
    assert np.all(np.abs(A.sum(1)) <= 1e-12 * scale)          # A_full 1 = 0
    assert np.linalg.eigvalsh(0.5 * (Aff + Aff.T)).min() > 0
    # every stored column is structurally present and columns are sorted
    for r in range(S["n_free"]):
        c = S["ff_col"][S["ff_row_ptr"][r]:S["ff_row_ptr"][r + 1]]
        assert np.all(np.diff(c) > 0)


def test_translation_invariance(orc, plain_sys):
    """Moving the mesh by a dyadic vector changes no class and no sample
    (counters do not depend on coordinates); the matrix agrees to rounding.
    The free mask is carried over (it is data, not recomputed)."""
    pb, S = plain_sys
    shift = np.array([0.5, -0.25, 0.125])
    m = pb.mesh
    T = orc.assemble(m.coords + shift, m.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                     g_nodal=pb.g_nodal)
    R = orc.assemble(m.coords, m.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                     g_nodal=pb.g_nodal)
    assert np.array_equal(T["pair_counts"], R["pair_counts"])
    for k in ["ff_row_ptr", "ff_col", "fc_row_ptr", "fc_col"]:
        assert np.array_equal(T[k], R[k]), k
    scale = np.abs(R["ff_val"]).max()
    assert np.max(np.abs(T["ff_val"] - R["ff_val"])) <= 1e-12 * scale
    assert np.max(np.abs(T["fc_val"] - R["fc_val"])) <= 1e-12 * scale
    assert np.max(np.abs(T["rhs"] - R["rhs"])) <= 1e-12 * np.abs(R["rhs"]).max()


def test_plain_cg_matches_dense_solve(orc, plain_sys):
    pb, S = plain_sys
    A = _dense(S, pb.mesh.n_vertices)[:, S["free_to_vertex"]]
    x, it, rr, rc = orc.cg(S["ff_row_ptr"], S["ff_col"], S["ff_val"], S["rhs"], rtol=1e-10)
    assert rc == 0 and rr <= 1e-10
    xd = np.linalg.solve(A, S["rhs"])
    assert np.max(np.abs(x - xd)) <= 1e-8 * np.max(np.abs(xd))


def _mass(mesh, weights=None):
    V = mesh.n_vertices
    M = np.zeros((V, V)); mv = np.zeros(V); vt = 0.0
    for e, t in enumerate(mesh.tets):
        X = mesh.coords[t]
        vol = abs(np.linalg.det(X[1:] - X[0])) / 6
        w = 1.0 if weights is None else weights[e]
        loc = vol / 20 * (np.ones((4, 4)) + np.eye(4))
        M[np.ix_(t, t)] += w * loc
        mv[t] += w * vol / 4
        vt += w * vol
    return M, mv, vt


def test_large_horizon_closed_form(orc):
    """delta larger than the mesh: every pair is IN and
    A_uv = psi (|O| M^f - m^O m^f^T - m^f m^O^T + M^O V^f), with M^O, m^O the P1 mass
    matrix / lumped mass over T_Omega tets (outer rule) and M^f, m^f, V^f the
    same over all tets weighted by 1 on T_Omega and 2 on T_Omega_I."""
    mesh = mg.kuhn_cube_mesh(2, jitter=0.15, seed=9)
    V, K = mesh.n_vertices, mesh.n_tets
    rng = np.random.default_rng(3)
    vfree = (rng.random(V) < 0.25).astype(np.uint8)
    region = np.array([1 if vfree[t].any() else int(rng.random() < 0.5) for t in mesh.tets], np.uint8)
    assert 0 < region.sum() < K and vfree.sum() > 0
    delta, psi = 10.0, 0.7
    S = orc.assemble(mesh.coords, mesh.tets, vfree, delta, psi, 8, 0, tet_region=region)
    assert S["pair_counts"][1:].sum() == 0
    MO, mO, VO = _mass(mesh, weights=region.astype(float))
    fw = np.where(region == 1, 1.0, 2.0)
    Mf, mf, Vf = _mass(mesh, weights=fw)
    Aexp = psi * (VO * Mf - np.outer(mO, mf) - np.outer(mf, mO) + MO * Vf)
    A = _dense(S, V)
    rows = S["free_to_vertex"]
    err = np.abs(A - Aexp[rows]).max()
    assert err <= 1e-12 * np.abs(Aexp).max(), err


def test_rhs_pins(orc):
    """f linear, g = 0 -> b_u = int over T_Omega of phi_u f = (M^O f_nodal)_u (the
    outer rule is exact for the quadratic phi_u f);
    f = 0, g = 1 -> the constant solves the system (L 1 = 0)."""
    pb = mg.plain_problem()
    m = pb.mesh
    K = m.n_tets
    lin = lambda x: 1.0 + 2.0 * x[..., 0] - 3.0 * x[..., 1] + 0.5 * x[..., 2]
    fq = np.array([[lin(orc.outer_point(m.coords, m.tets, n, k)) for k in range(4)] for n in range(K)])
    S1 = orc.assemble(m.coords, m.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                      f_qp=fq, g_nodal=np.zeros(m.n_vertices))
    region = np.array([pb.vertex_free[t].any() for t in m.tets], float)
    MO, _, _ = _mass(m, weights=region)
    bexp = MO @ lin(m.coords)
    assert np.allclose(S1["rhs"], bexp[S1["free_to_vertex"]], rtol=1e-13, atol=1e-14 * np.abs(bexp).max())
    S2 = orc.assemble(m.coords, m.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                      f_qp=np.zeros((K, 4)), g_nodal=np.ones(m.n_vertices))
    x, it, rr, rc = orc.cg(S2["ff_row_ptr"], S2["ff_col"], S2["ff_val"], S2["rhs"], rtol=1e-12)
    assert rc == 0
    assert np.max(np.abs(x - 1.0)) < 1e-9


def test_pair_counts_match_pointwise_brute_force(orc, plain_sys):
    """The assembly's pair class counts equal the per-point brute-force classification."""
    pb, S = plain_sys
    m = pb.mesh
    region = np.array([pb.vertex_free[t].any() for t in m.tets])
    counts = np.zeros(5, np.int64)
    for n in np.nonzero(region)[0]:
        for k in range(4):
            p = orc.outer_point(m.coords, m.tets, int(n), k)
            cls = orc.classify_point(m.coords, m.tets, pb.delta, p)
            counts[0] += np.sum(cls == 1)
            for c in range(4):
                counts[1 + c] += np.sum(cls == 2 + c)
    assert np.array_equal(counts, S["pair_counts"])
