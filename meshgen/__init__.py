"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only builds meshes and data fields; it contains none of the
assembly arithmetic.  Everything here is deterministic given its seeds.

* Kuhn-split cube meshes of [0,1]^3: each of the n^3 cubes is split into the
  6 tetrahedra (c, c+e_s1, c+e_s1+e_s2, c+(1,1,1)) over the permutations s of
  the axes, which gives a conforming mesh with h = 1/n.  The paper measures on
  unstructured tetrahedral meshes of the unit cube (Sec. 5, 3D experiment);
  those meshes are not available, so jittered Kuhn meshes stand in for them.
* Interior-vertex jitter: every vertex strictly inside the cube moves by an
  independent uniform offset in [-J h, J h] per coordinate (numpy PCG64 seeded
  stream).  Boundary vertices stay put, so the domain is still the unit cube.
  With J <= 0.25 no tetrahedron can invert (minimum Kuhn height is h/sqrt(2)).
* Volume constraint: a vertex is a free unknown iff its distance to the cube
  boundary is larger than delta (nodes within delta of the boundary, and on it,
  carry the nonlocal Dirichlet data; Sec. 3.2, node assignment rule).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# the six permutations of (x, y, z) in lexicographic order
_PERMS = list(itertools.permutations(range(3)))


@dataclass
class Mesh:
    coords: np.ndarray          # float64 [V, 3]
    tets: np.ndarray            # int32   [K, 4]
    n: int = 0                  # cubes per side (0 for hand-built meshes)
    h: float = 0.0              # cube side
    info: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


def kuhn_cube_mesh(n: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Kuhn-split n x n x n cube mesh of [0,1]^3.

    Vertex id = i + (n+1) (j + (n+1) k); tet id = 6 * cube_id + perm index with
    cube_id = i + n (j + n k).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) / n
    kk, jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    ii = ii.reshape(-1); jj = jj.reshape(-1); kk = kk.reshape(-1)
    coords = np.stack([g[ii], g[jj], g[kk]], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        interior = (ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)
        coords[interior] += off[interior]

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
    return Mesh(coords=coords, tets=tets.reshape(-1, 4).astype(np.int32), n=n, h=h,
                info={"kind": "kuhn", "n": n, "jitter": jitter, "seed": seed})


def single_tet_mesh(scale: float = 1.0) -> Mesh:
    """One right-angled tetrahedron with legs `scale`."""
    coords = np.array([[0, 0, 0], [scale, 0, 0], [0, scale, 0], [0, 0, scale]], dtype=np.float64)
    return Mesh(coords=coords, tets=np.array([[0, 1, 2, 3]], dtype=np.int32), info={"kind": "single"})


def tet_mesh(points) -> Mesh:
    """One tetrahedron with the given 4 vertices."""
    coords = np.asarray(points, dtype=np.float64).reshape(4, 3)
    return Mesh(coords=coords, tets=np.array([[0, 1, 2, 3]], dtype=np.int32), info={"kind": "single"})


def six_tet_cube_mesh(side: float = 1.0) -> Mesh:
    """The unit cube (scaled) split into the 6 Kuhn tetrahedra."""
    m = kuhn_cube_mesh(1)
    m.coords *= side
    m.h = side
    m.info["kind"] = "six_tet"
    return m


def free_mask_box(coords: np.ndarray, delta: float) -> np.ndarray:
    """1 where min(x, 1-x, y, 1-y, z, 1-z) > delta (a free unknown), else 0."""
    c = np.asarray(coords, dtype=np.float64)
    d = np.minimum(c, 1.0 - c).min(axis=1)
    return (d > delta).astype(np.uint8)


def g_x1_squared(coords: np.ndarray) -> np.ndarray:
    """Nodal volume-constraint data g = x1^2."""
    return np.ascontiguousarray(coords[:, 0] * coords[:, 0], dtype=np.float64)


def const_f_qp(n_tets: int, value: float) -> np.ndarray:
    """Constant source f at the 4 outer quadrature points of every tet."""
    return np.full((n_tets, 4), value, dtype=np.float64)


def psi_unit_laplacian(delta: float) -> float:
    """Kernel constant psi with int_B psi |z|^2 dz = 3 in 3D, i.e. with the
    paper's operator L u = 2 int_B (u(y)-u(x)) psi dy this gives L x1^2 = 2."""
    return 15.0 / (4.0 * math.pi * delta ** 5)


@dataclass
class Problem:
    """One assemble(+CG) request: mesh, fields and parameters."""
    name: str
    mesh: Mesh
    delta: float
    psi: float
    mc_samples: int
    seed: int
    vertex_free: np.ndarray
    f_qp: np.ndarray
    g_nodal: np.ndarray
    precision: str = "fp64"     # "fp64" or "fp32"
    info: dict = field(default_factory=dict)
    strategy: str = "fullcaps"  # ball approximation: fullcaps, nocaps, overlap, inside, barycenter
    cap_sampling: str = "whole"  # cap samples on the whole element, or on E_m minus U_I ("outside_ui")
    tet_region: np.ndarray | None = None  # explicit T_Omega mask; None: tets with a free vertex
    g_poly: np.ndarray | None = None  # g as tensor coefficients [a, b, c] of y1^a y2^b y3^c, when known
    keying: str = "pair"  # Monte Carlo samples per (point, element) pair ("pair") or per element ("element")


def make_problem(name: str, n: int, delta_over_h: float | None = None, delta: float | None = None,
                 jitter: float = 0.0, jitter_seed: int = 0, mc_samples: int = 32, seed: int = 0,
                 f_value: float = -2.0, precision: str = "fp64") -> Problem:
    mesh = kuhn_cube_mesh(n, jitter=jitter, seed=jitter_seed)
    if delta is None:
        delta = float(delta_over_h) / n
    return Problem(name=name, mesh=mesh, delta=delta, psi=psi_unit_laplacian(delta),
                   mc_samples=mc_samples, seed=seed,
                   vertex_free=free_mask_box(mesh.coords, delta),
                   f_qp=const_f_qp(mesh.n_tets, f_value), g_nodal=g_x1_squared(mesh.coords),
                   precision=precision,
                   info={"n": n, "delta_over_h": delta * n, "jitter": jitter, "jitter_seed": jitter_seed})


# --- the five workload families -------------------------------------------------

def plain_problem() -> Problem:
    """6x6x6 Kuhn cubes (1296 tets, 343 vertices), delta = 0.25, N = 32, seed 0."""
    return make_problem("plain", 6, delta=0.25, mc_samples=32, seed=0)


def precision_problem(precision: str = "fp64") -> Problem:
    """32^3 Kuhn cubes (196,608 tets), jitter 0.2h (seed 1), delta = 3h, N = 64."""
    return make_problem("precision", 32, delta_over_h=3.0, jitter=0.2, jitter_seed=1,
                        mc_samples=64, seed=0, precision=precision)


def large_problem() -> Problem:
    """64^3 Kuhn cubes (1,572,864 tets), jitter 0.2h (seed 1), delta = 4h, N = 128."""
    return make_problem("large", 64, delta_over_h=4.0, jitter=0.2, jitter_seed=1,
                        mc_samples=128, seed=0, precision="fp32")


def batched_problems(count: int = 256, precision: str = "fp32") -> list[Problem]:
    """Uneven batch: n ~ U{8..24}, delta/h ~ U{2,3,4}, jitter 0.15h (seed 1000+b),
    N = 32, MC seed b.  (n, delta/h) drawn from a seed-2 stream."""
    rng = np.random.default_rng(2)
    ns = rng.integers(8, 25, size=count)
    rs = rng.choice([2, 3, 4], size=count)
    out = []
    for b in range(count):
        out.append(make_problem(f"batch{b}", int(ns[b]), delta_over_h=float(rs[b]), jitter=0.15,
                                jitter_seed=1000 + b, mc_samples=32, seed=b, precision=precision))
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    problem: Problem


def serving_requests(count: int = 500, rate_per_s: float = 50.0, n_max: int = 40,
                     seed: int = 3) -> list[Request]:
    """Poisson arrivals; n ~ U{8..n_max}, delta/h ~ U[2,5], N in {32, 64},
    precision fp64/fp32 50/50, jitter 0.15h; per-request seeds = request id."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(8, n_max + 1, size=count)
    rs = rng.uniform(2.0, 5.0, size=count)
    nmc = rng.choice([32, 64], size=count)
    prec = rng.choice(["fp64", "fp32"], size=count)
    out = []
    for r in range(count):
        pb = make_problem(f"req{r}", int(ns[r]), delta_over_h=float(rs[r]), jitter=0.15,
                          jitter_seed=10000 + r, mc_samples=int(nmc[r]), seed=r, precision=str(prec[r]))
        out.append(Request(rid=r, arrival_s=float(t[r]), problem=pb))
    return out


def outer_subset_mask(n_tets: int, fraction: float, seed: int = 7) -> np.ndarray:
    """Deterministic subset of outer tets (1 = assemble this outer tet)."""
    rng = np.random.default_rng(seed)
    return (rng.random(n_tets) < fraction).astype(np.uint8)


from .convergence import convergence_problem  # noqa: E402  (the convergence workload)
