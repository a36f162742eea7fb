"""Python access to the serial FP64 oracle (test infrastructure only).

The oracle is the checker: only tests, the smoke check and the CPU-baseline
leg of the benchmark load it.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlfem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CLS_OUT, CLS_IN, CLS_CUT0 = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrProblem(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_tets", C.c_int64),
                ("coords", C.c_void_p), ("tets", C.c_void_p), ("vertex_free", C.c_void_p),
                ("tet_region", C.c_void_p), ("delta", C.c_double), ("psi", C.c_double),
                ("mc_samples", C.c_int32), ("seed", C.c_uint64), ("outer_mask", C.c_void_p),
                ("f_qp", C.c_void_p), ("g_nodal", C.c_void_p), ("strategy", C.c_int32),
                ("cap_sampling", C.c_int32), ("g_degree", C.c_int32), ("g_coef", C.c_void_p),
                ("keying", C.c_int32)]


# ball approximation strategies (Sec. 4.1), as numbered in the oracle
STRATEGIES = {"fullcaps": 0, "nocaps": 1, "overlap": 2, "inside": 3, "barycenter": 4}


def _strategy(st):
    return STRATEGIES[st] if isinstance(st, str) else int(st)


CAP_SAMPLING = {"whole": 0, "outside_ui": 1}


def _caps(cs):
    return CAP_SAMPLING[cs] if isinstance(cs, str) else int(cs)


# Monte Carlo sample keying: N samples per (point, element) pair, or per element
KEYING = {"pair": 0, "element": 1}


def _key(kk):
    return KEYING[kk] if isinstance(kk, str) else int(kk)


class OrSystem(C.Structure):
    _fields_ = [("n_free", C.c_int64), ("nnz_ff", C.c_int64), ("nnz_fc", C.c_int64),
                ("ff_row_ptr", C.POINTER(C.c_int64)), ("ff_col", C.POINTER(C.c_int32)),
                ("ff_val", C.POINTER(C.c_double)),
                ("fc_row_ptr", C.POINTER(C.c_int64)), ("fc_col", C.POINTER(C.c_int32)),
                ("fc_val", C.POINTER(C.c_double)),
                ("rhs", C.POINTER(C.c_double)), ("free_to_vertex", C.POINTER(C.c_int32)),
                ("pair_counts", C.c_int64 * 5), ("near_ties", C.c_int64),
                ("tie_allow", C.POINTER(C.c_double)), ("tie_allow_rhs", C.POINTER(C.c_double))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        # NLFEM_ORACLE_LIB: a copy of the oracle built elsewhere (the mutation
        # tests point it at copies with a planted mistake)
        L = C.CDLL(os.environ.get("NLFEM_ORACLE_LIB") or _LIB)
        P = C.c_void_p
        L.or_rule_constants.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_sample_lambda.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P]
        L.or_sample_lambda_keyed.argtypes = [C.c_uint64, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, P]
        L.or_pair_moments_keyed.argtypes = [P, P, C.c_int64, C.c_int, C.c_int64, C.c_double, C.c_int,
                                            C.c_uint64, C.c_int, C.c_int, C.c_int, P, P]
        L.or_pair_moments_keyed.restype = C.c_int
        L.or_point_moments_keyed.argtypes = [P, P, C.c_int64, C.c_int64, C.c_int, C.c_double, C.c_int,
                                             C.c_uint64, C.c_int, C.c_int, C.c_int, P, P, P]
        L.or_pair_samples.argtypes = [P, P, C.c_int64, C.c_int, C.c_int64, C.c_double, C.c_int, C.c_uint64,
                                      C.c_int, C.c_int, P, P, P]
        L.or_pair_samples.restype = C.c_int
        L.or_outer_point.argtypes = [P, P, C.c_int64, C.c_int, P]
        L.or_classify_point.argtypes = [P, P, C.c_int64, C.c_double, P, P]
        L.or_pair_moments.argtypes = [P, P, C.c_int64, C.c_int, C.c_int64, C.c_double, C.c_int,
                                      C.c_uint64, C.c_int, C.c_int, P]
        L.or_pair_moments.restype = C.c_int
        L.or_point_moments.argtypes = [P, P, C.c_int64, C.c_int64, C.c_int, C.c_double, C.c_int,
                                       C.c_uint64, C.c_int, C.c_int, P, P]
        L.or_pair_geometry.argtypes = [P, P, C.c_int64, C.c_int, C.c_int64, C.c_double, P, P, P, P,
                                       P, P, P]
        L.or_pair_geometry.restype = C.c_int
        L.or_cap_region.argtypes = [P, P, C.c_int64, C.c_int, C.c_int64, C.c_double, P, P]
        L.or_cap_region.restype = C.c_int
        L.or_assemble.argtypes = [C.POINTER(OrProblem), C.POINTER(OrSystem)]
        L.or_assemble.restype = C.c_int
        L.or_system_free.argtypes = [C.POINTER(OrSystem)]
        L.or_cg.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, C.c_int32,
                            C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.or_cg.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def rule_constants():
    a, b = C.c_double(), C.c_double()
    lib().or_rule_constants(C.byref(a), C.byref(b))
    return a.value, b.value


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sample_lambda(seed, q, m, s, keying="pair"):
    lam = np.zeros(4)
    lib().or_sample_lambda_keyed(seed, _key(keying), q, m, s, _p(lam))
    return lam


def outer_point(coords, tets, n, k):
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    p = np.zeros(3)
    lib().or_outer_point(_p(coords), _p(tets), n, k, _p(p))
    return p


def classify_point(coords, tets, delta, p):
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    p = _c(p, np.float64)
    out = np.zeros(tets.shape[0], dtype=np.int8)
    lib().or_classify_point(_p(coords), _p(tets), tets.shape[0], delta, _p(p), _p(out))
    return out


def pair_moments(coords, tets, n, k, m, delta, N, seed, strategy="fullcaps", cap_sampling="whole",
                 keying="pair", with_ties=False):
    """(class, S[15]) of pair (4 n + k, m); with_ties: (class, S, near ties)."""
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    S = np.zeros(15)
    ties = C.c_int32()
    cls = lib().or_pair_moments_keyed(_p(coords), _p(tets), n, k, m, delta, N, seed, _strategy(strategy),
                                      _caps(cap_sampling), _key(keying), _p(S), C.byref(ties))
    return (cls, S, ties.value) if with_ties else (cls, S)


def point_moments(coords, tets, n, k, delta, N, seed, strategy="fullcaps", cap_sampling="whole",
                  keying="pair", with_ties=False):
    """Classes [K] and moments [K, 15] of outer point 4 n + k against every
    tet; with_ties: also the near-tie count of each pair's samples."""
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    K = tets.shape[0]
    cls = np.zeros(K, dtype=np.int8)
    S = np.zeros((K, 15))
    ties = np.zeros(K, dtype=np.int32)
    lib().or_point_moments_keyed(_p(coords), _p(tets), K, n, k, delta, N, seed, _strategy(strategy),
                                 _caps(cap_sampling), _key(keying), _p(cls), _p(S), _p(ties))
    return (cls, S, ties) if with_ties else (cls, S)


def pair_samples(coords, tets, n, k, m, delta, N, seed, cap_sampling="whole", keying="pair"):
    """Per Monte Carlo sample of pair (4 n + k, m): |y - p|^2 as the oracle's
    sample test evaluates it, accepted, near tie.  (class, rr, acc, tie)."""
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    rr = np.full(N, np.nan)
    acc = np.zeros(N, dtype=np.int8)
    tie = np.zeros(N, dtype=np.int8)
    cls = lib().or_pair_samples(_p(coords), _p(tets), n, k, m, delta, N, seed, _caps(cap_sampling), _key(keying),
                                _p(rr), _p(acc), _p(tie))
    return cls, rr, acc.astype(bool), tie.astype(bool)


def pair_geometry(coords, tets, n, k, m, delta):
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    t = np.zeros(16); sub = np.zeros(48); subvol = np.zeros(3); plane = np.zeros(8)
    ns, npl, split = C.c_int(), C.c_int(), C.c_int()
    nin = lib().or_pair_geometry(_p(coords), _p(tets), n, k, m, delta, _p(t), _p(sub), _p(subvol),
                                 _p(plane), C.byref(ns), C.byref(npl), C.byref(split))
    return {"n_in": nin, "t": t.reshape(4, 4), "sub": sub.reshape(3, 4, 4)[:max(ns.value, 0)],
            "subvol": subvol[:max(ns.value, 0)], "planes": plane.reshape(2, 4)[:max(npl.value, 0)],
            "split": split.value}


def cap_region(coords, tets, n, k, m, delta):
    """Sub-tets of the cap region E - U_I of pair (4 n + k, m) as sampled with
    cap sampling on: (rows [j, 4, 4] barycentric in E, point 0 the apex, and
    volumes [j]); None when the pair is not cut, no sub-tets for CUT(0)."""
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    rows = np.zeros(48); vol = np.zeros(3)
    n_sub = lib().or_cap_region(_p(coords), _p(tets), n, k, m, delta, _p(rows), _p(vol))
    if n_sub < 0:
        return None
    return rows.reshape(3, 4, 4)[:n_sub], vol[:n_sub]


def gpoly_coef(g_poly):
    """[a, b, c] array of the coefficients of y1^a y2^b y3^c -> (degree, flat
    array with index a + n1 (b + n1 c))."""
    G = np.asarray(g_poly, dtype=np.float64)
    n1 = G.shape[0]
    assert G.shape == (n1, n1, n1)
    return n1 - 1, np.ascontiguousarray(G.transpose(2, 1, 0)).reshape(-1)


def assemble(coords, tets, vertex_free, delta, psi, mc_samples, seed, f_qp=None, g_nodal=None,
             tet_region=None, outer_mask=None, strategy="fullcaps", cap_sampling="whole", g_poly=None,
             keying="pair"):
    """Full oracle assembly.  Returns a dict of numpy arrays (CSR blocks + rhs)
    and the near-tie report (near_ties; tie_allow / tie_allow_rhs per free row).
    With g_poly (tensor coefficients [a, b, c]) the right-hand side uses g
    itself inside the inner integrals over Omega_I (eqs. Fh, F1.5)."""
    coords = _c(coords, np.float64); tets = _c(tets, np.int32)
    vf = _c(vertex_free, np.uint8); tr = _c(tet_region, np.uint8); om = _c(outer_mask, np.uint8)
    fq = _c(f_qp, np.float64); gn = _c(g_nodal, np.float64)
    gdeg, gc = (0, None) if g_poly is None else gpoly_coef(g_poly)
    P = OrProblem(coords.shape[0], tets.shape[0], _p(coords), _p(tets), _p(vf), _p(tr), delta, psi,
                  mc_samples, seed, _p(om), _p(fq), _p(gn), _strategy(strategy), _caps(cap_sampling),
                  gdeg, _p(gc), _key(keying))
    S = OrSystem()
    rc = lib().or_assemble(C.byref(P), C.byref(S))
    if rc != 0:
        raise RuntimeError(f"oracle assemble failed rc={rc}")
    try:
        nf = S.n_free

        def arr(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt, copy=True)
        out = {
            "n_free": nf,
            "ff_row_ptr": arr(S.ff_row_ptr, nf + 1, np.int64),
            "ff_col": arr(S.ff_col, S.nnz_ff, np.int32),
            "ff_val": arr(S.ff_val, S.nnz_ff, np.float64),
            "fc_row_ptr": arr(S.fc_row_ptr, nf + 1, np.int64),
            "fc_col": arr(S.fc_col, S.nnz_fc, np.int32),
            "fc_val": arr(S.fc_val, S.nnz_fc, np.float64),
            "rhs": arr(S.rhs, nf, np.float64),
            "free_to_vertex": arr(S.free_to_vertex, nf, np.int32),
            "pair_counts": np.array(list(S.pair_counts), dtype=np.int64),
            "near_ties": int(S.near_ties),
            "tie_allow": arr(S.tie_allow, nf, np.float64),
            "tie_allow_rhs": arr(S.tie_allow_rhs, nf, np.float64),
        }
        if nf == 0:
            out["ff_row_ptr"] = np.zeros(1, dtype=np.int64)
            out["fc_row_ptr"] = np.zeros(1, dtype=np.int64)
    finally:
        lib().or_system_free(C.byref(S))
    return out


def cg(row_ptr, col, val, b, rtol=1e-10, max_iter=None, x0=None):
    n = len(b)
    rp = _c(row_ptr, np.int64); ci = _c(col, np.int32); va = _c(val, np.float64)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    it, rr = C.c_int32(), C.c_double()
    rc = lib().or_cg(n, _p(rp), _p(ci), _p(va), _p(bb), _p(x), rtol,
                     n if max_iter is None else max_iter, C.byref(it), C.byref(rr))
    return x, it.value, rr.value, rc


def problem_assemble(pb, outer_mask=None, exact_g=False):
    m = pb.mesh
    return assemble(m.coords, m.tets, pb.vertex_free, pb.delta, pb.psi, pb.mc_samples, pb.seed,
                    f_qp=pb.f_qp, g_nodal=pb.g_nodal, outer_mask=outer_mask,
                    g_poly=pb.g_poly if exact_g else None,
                    tet_region=getattr(pb, "tet_region", None),
                    strategy=getattr(pb, "strategy", "fullcaps"),
                    cap_sampling=getattr(pb, "cap_sampling", "whole"),
                    keying=getattr(pb, "keying", "pair"))
