"""Convergence workload: the paper's 3D accuracy experiment (Sec. 5, 3D
numerical experiments) on synthetic meshes.

Omega = (0,1)^3, delta = 0.1, constant kernel on the ball, manufactured
solution u(x) = x1 (1-x1) x2 (1-x2) x3 (1-x3).  The paper's meshes are not
available; Kuhn-split cube meshes of the box Omega plus a collar of whole
cubes at least delta wide stand in for them, refined by cubes per unit length
m (h = 1/m), with the vertices strictly inside Omega jittered.

Everything here is problem data (mesh, u, f = -L u at the outer quadrature
points, g = u at the vertices) or measurement (the L2 error of a P1 field
against u); none of it is the assembly.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_jacobi

from . import Mesh, Problem, _PERMS

# ---------------------------------------------------------------------------
# mesh


def collar_cubes(m: int, delta: float) -> int:
    """Whole cubes of side 1/m that cover a collar at least delta wide."""
    c = int(math.ceil(delta * m - 1e-12))
    return max(c, 1)


def box_kuhn_mesh(m: int, collar: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Kuhn-split cubes of side h = 1/m covering [-collar h, 1 + collar h]^3.

    Vertex (i, j, k) sits at ((i - collar)/m, (j - collar)/m, (k - collar)/m),
    so the planes x_d = 0 and x_d = 1 are mesh faces exactly.  Vertices with
    all three indices strictly between collar and collar + m (strictly inside
    (0,1)^3) move by an independent uniform offset in [-J h, J h] per
    coordinate (PCG64 stream `seed`); the others stay on the grid, so the mesh
    still conforms to the boundary of (0,1)^3.  Tet order as kuhn_cube_mesh.
    """
    if m < 1 or collar < 1:
        raise ValueError("m and collar must be >= 1")
    n = m + 2 * collar
    idx = np.arange(n + 1)
    kk, jj, ii = np.meshgrid(idx, idx, idx, indexing="ij")
    ii = ii.reshape(-1); jj = jj.reshape(-1); kk = kk.reshape(-1)
    coords = np.stack([(ii - collar) / m, (jj - collar) / m, (kk - collar) / m], axis=1).astype(np.float64)
    inside = ((ii > collar) & (ii < collar + m) & (jj > collar) & (jj < collar + m)
              & (kk > collar) & (kk < collar + m))
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter / m, jitter / m, size=coords.shape)
        coords[inside] += off[inside]

    def vid(i, j, k):
        return i + (n + 1) * (j + (n + 1) * k)

    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.reshape(-1); cj = cj.reshape(-1); ck = ck.reshape(-1)
    base = np.stack([ci, cj, ck], axis=1)
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        cur = base.copy()
        tets[:, p, 0] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
        for s in range(3):
            cur[:, perm[s]] += 1
            tets[:, p, s + 1] = vid(cur[:, 0], cur[:, 1], cur[:, 2])
    in_omega = ((ci >= collar) & (ci < collar + m) & (cj >= collar) & (cj < collar + m)
                & (ck >= collar) & (ck < collar + m))
    mesh = Mesh(coords=coords, tets=tets.reshape(-1, 4).astype(np.int32), n=n, h=1.0 / m,
                info={"kind": "box_kuhn", "m": m, "collar": collar, "jitter": jitter, "seed": seed})
    mesh.info["vertex_inside"] = inside.astype(np.uint8)
    mesh.info["tet_in_omega"] = np.repeat(in_omega, 6).astype(np.uint8)
    return mesh


# ---------------------------------------------------------------------------
# manufactured solution and source


def u_exact(x: np.ndarray) -> np.ndarray:
    """u(x) = x1 (1-x1) x2 (1-x2) x3 (1-x3) (Sec. 5, 3D experiment)."""
    x = np.asarray(x, dtype=np.float64)
    q = x * (1.0 - x)
    return q[..., 0] * q[..., 1] * q[..., 2]


def u_tensor_coef() -> np.ndarray:
    """u as tensor coefficients G[a, b, c] of y1^a y2^b y3^c: the product of
    x (1 - x) = x - x^2 in each coordinate."""
    q = np.array([0.0, 1.0, -1.0])
    return np.einsum("a,b,c->abc", q, q, q)


def ball_even_moments(delta: float) -> tuple[float, float, float, float]:
    """|B|, int_B z1^2, int_B z1^2 z2^2, int_B z1^2 z2^2 z3^2 over the ball of
    radius delta (radial integral times the sphere averages 1/3, 1/15, 1/105)."""
    d = float(delta)
    return (4.0 * math.pi * d ** 3 / 3.0, 4.0 * math.pi * d ** 5 / 15.0,
            4.0 * math.pi * d ** 7 / 105.0, 4.0 * math.pi * d ** 9 / 945.0)


def f_exact(x: np.ndarray, delta: float, psi: float) -> np.ndarray:
    """f = -L u with L v(x) = 2 psi int_{B_delta(x)} (v(y) - v(x)) dy.

    With a_d = x_d (1 - x_d), u(x + z) = prod_d (a_d + (1 - 2 x_d) z_d - z_d^2);
    over the ball the odd powers of every z_d integrate to zero, so
    int_B (u(x+z) - u(x)) dz = -s2 M2 + s1 M22 - M222 with s1 = sum a_d,
    s2 = sum_{d<e} a_d a_e and the even moments of ball_even_moments.
    """
    x = np.asarray(x, dtype=np.float64)
    a = x * (1.0 - x)
    s1 = a[..., 0] + a[..., 1] + a[..., 2]
    s2 = a[..., 0] * a[..., 1] + a[..., 0] * a[..., 2] + a[..., 1] * a[..., 2]
    _, m2, m22, m222 = ball_even_moments(delta)
    return -2.0 * psi * (-s2 * m2 + s1 * m22 - m222)


# the degree-2, 4-point rule of the outer integral (Sec. 4.2.1): point k has
# barycentric weight ALPHA on vertex k and BETA on the other three
ALPHA = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
BETA = (5.0 - math.sqrt(5.0)) / 20.0


def outer_rule_points(coords: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """[K, 4, 3]: the 4 outer quadrature points of every tet."""
    X = np.asarray(coords, dtype=np.float64)[np.asarray(tets)]
    s = X.sum(axis=1, keepdims=True)
    return ALPHA * X + BETA * (s - X)


# ---------------------------------------------------------------------------
# the workload


def convergence_problem(m: int, delta: float = 0.1, mc_samples: int = 64, seed: int = 0,
                        jitter: float = 0.1, jitter_seed: int = 11, strategy: str = "fullcaps",
                        precision: str = "fp64") -> Problem:
    """Omega = (0,1)^3 with h = 1/m, delta = 0.1: free vertices strictly inside
    Omega, T_Omega = the tets of Omega (explicit region), f = -L u at the outer
    quadrature points, g = u at every vertex."""
    from . import psi_unit_laplacian
    collar = collar_cubes(m, delta)
    mesh = box_kuhn_mesh(m, collar, jitter=jitter, seed=jitter_seed + m)
    psi = psi_unit_laplacian(delta)
    f_qp = np.ascontiguousarray(f_exact(outer_rule_points(mesh.coords, mesh.tets), delta, psi))
    pb = Problem(name=f"convergence_m{m}", mesh=mesh, delta=float(delta), psi=psi, mc_samples=mc_samples,
                 seed=seed, vertex_free=mesh.info["vertex_inside"].copy(), f_qp=f_qp,
                 g_nodal=np.ascontiguousarray(u_exact(mesh.coords)), precision=precision,
                 info={"m": m, "h": 1.0 / m, "collar": collar, "delta_over_h": delta * m, "jitter": jitter},
                 strategy=strategy)
    pb.tet_region = mesh.info["tet_in_omega"].copy()
    pb.g_poly = u_tensor_coef()
    return pb


# ---------------------------------------------------------------------------
# measurement: L2(Omega) error of a P1 field


def tet_rule(n: int = 4) -> tuple[np.ndarray, np.ndarray]:
    """Collapsed (conical product) Gauss-Jacobi rule on the reference tet
    {xi >= 0, xi1 + xi2 + xi3 <= 1}: n^3 points, exact for polynomials of
    total degree 2n - 1.  Returns barycentrics [n^3, 4] (lambda_0 = 1 - sum xi)
    and weights [n^3] that sum to 1 (the tet's volume factors out)."""
    ra, wa = roots_jacobi(n, 2.0, 0.0)   # weight (1-t)^2 on [-1,1]
    rb, wb = roots_jacobi(n, 1.0, 0.0)   # weight (1-t)
    rc, wc = roots_jacobi(n, 0.0, 0.0)   # Gauss-Legendre
    a = (ra + 1.0) / 2.0; b = (rb + 1.0) / 2.0; c = (rc + 1.0) / 2.0
    wa = wa / 8.0; wb = wb / 4.0; wc = wc / 2.0
    A, B, Cc = np.meshgrid(a, b, c, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]).reshape(-1)
    x1 = A.reshape(-1)
    x2 = (B * (1.0 - A)).reshape(-1)
    x3 = (Cc * (1.0 - A) * (1.0 - B)).reshape(-1)
    lam = np.stack([1.0 - x1 - x2 - x3, x1, x2, x3], axis=1)
    return lam, W / W.sum()


def l2_error(coords: np.ndarray, tets: np.ndarray, tet_mask: np.ndarray, nodal: np.ndarray,
             u=u_exact, n: int = 4, chunk: int = 65536) -> float:
    """|| sum_v nodal_v phi_v - u ||_{L2} over the tets where tet_mask is 1."""
    coords = np.asarray(coords, dtype=np.float64)
    sel = np.nonzero(np.asarray(tet_mask))[0]
    lam, w = tet_rule(n)
    tot = 0.0
    for s in range(0, len(sel), chunk):
        T = np.asarray(tets)[sel[s:s + chunk]]
        X = coords[T]                                   # [c, 4, 3]
        vol = np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6.0
        pts = np.einsum("qj,cjd->cqd", lam, X)           # [c, q, 3]
        uh = np.asarray(nodal, dtype=np.float64)[T] @ lam.T   # [c, q]
        e = uh - u(pts)
        tot += float(np.sum(vol * (e * e @ w)))
    return math.sqrt(tot)
