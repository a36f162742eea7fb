"""Comparison helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def pattern_equal(g, o):
    """CSR patterns must be identical (canonical ordering on both sides)."""
    assert g["n_free"] == o["n_free"]
    for k in ["ff_row_ptr", "ff_col", "fc_row_ptr", "fc_col", "free_to_vertex"]:
        assert np.array_equal(np.asarray(g[k]), np.asarray(o[k])), k


def row_scale(S):
    """max |A_uv| over each full row (free and constrained columns)."""
    nf = S["n_free"]
    sc = np.zeros(nf)
    for blk in ["ff", "fc"]:
        rp, v = S[blk + "_row_ptr"], np.abs(S[blk + "_val"])
        for r in range(nf):
            if rp[r + 1] > rp[r]:
                sc[r] = max(sc[r], v[rp[r]:rp[r + 1]].max())
    return sc


def value_errors(g, o):
    """Per-entry errors: (max abs error / row scale, max rel error on entries
    above 1e-6 of the row scale), rhs relative error.  Where the oracle reports
    near ties of its Monte Carlo sample test (samples a different evaluation
    order may decide the other way), each entry's difference is first reduced
    by the most those samples can move it (o["tie_allow"] per row), so only
    the rest is compared; o["near_ties"] is passed through."""
    sc = row_scale(o)
    nf = o["n_free"]
    allow = np.asarray(o.get("tie_allow", np.zeros(nf)))
    allow_rhs = np.asarray(o.get("tie_allow_rhs", np.zeros(nf)))
    out = {"near_ties": int(o.get("near_ties", 0))}
    for blk in ["ff", "fc"]:
        rp = o[blk + "_row_ptr"]
        rows = np.repeat(np.arange(o["n_free"]), np.diff(rp))
        a, b = np.asarray(g[blk + "_val"]), np.asarray(o[blk + "_val"])
        if len(b) == 0:
            out[blk + "_abs"] = 0.0
            out[blk + "_rel"] = 0.0
            continue
        d = np.maximum(np.abs(a - b) - allow[rows], 0.0)
        s = np.maximum(sc[rows], 1e-300)
        out[blk + "_abs"] = float(np.max(d / s))
        big = np.abs(b) > 1e-6 * s
        out[blk + "_rel"] = float(np.max(d[big] / np.abs(b[big]))) if big.any() else 0.0
    rb = np.asarray(o["rhs"])
    if len(rb):
        dr = np.maximum(np.abs(np.asarray(g["rhs"]) - rb) - allow_rhs, 0.0)
        out["rhs"] = float(np.max(dr) / max(np.max(np.abs(rb)), 1e-300))
    else:
        out["rhs"] = 0.0
    return out


def row_sums(S):
    """A_full 1 per free row and the matching scale sum |A_uv|."""
    nf = S["n_free"]
    tot = np.zeros(nf)
    mag = np.zeros(nf)
    for blk in ["ff", "fc"]:
        rp, v = S[blk + "_row_ptr"], S[blk + "_val"]
        rows = np.repeat(np.arange(nf), np.diff(rp))
        np.add.at(tot, rows, v)
        np.add.at(mag, rows, np.abs(v))
    return tot, mag


def dense_ff(S):
    nf = S["n_free"]
    A = np.zeros((nf, nf))
    rp = S["ff_row_ptr"]
    for r in range(nf):
        A[r, S["ff_col"][rp[r]:rp[r + 1]]] = S["ff_val"][rp[r]:rp[r + 1]]
    return A


def sparse_ff(S):
    import scipy.sparse as sp
    nf = S["n_free"]
    return sp.csr_matrix((S["ff_val"], S["ff_col"], S["ff_row_ptr"]), shape=(nf, nf))


def moment_errors(Sg, So, ties, weight):
    """Per-pair moments of the library (Sg [P, 15]) against the oracle's (So),
    relative to each pair's largest moment.  A pair with near ties of the
    sample test (ties [P]) may differ by the largest sample weight (weight [P])
    of each such sample in every moment (all moment integrands lie in [0, 1]);
    that much is taken off first.  Returns the largest remaining error."""
    Sg, So = np.asarray(Sg), np.asarray(So)
    if len(So) == 0:
        return 0.0
    allow = (np.asarray(ties, dtype=float) * np.asarray(weight, dtype=float))[:, None]
    scale = np.maximum(np.abs(So).max(axis=1, keepdims=True), 1e-300)
    d = np.maximum(np.abs(Sg - So) - allow, 0.0)
    return float(np.max(d / scale))


def tet_volumes(coords, tets):
    X = np.asarray(coords)[np.asarray(tets)]
    return np.abs(np.linalg.det(X[:, 1:] - X[:, :1])) / 6.0


def point_pairs_vs_oracle(orc, mesh, rec, n, k, delta, N, seed, strategy="fullcaps", cap_sampling="whole",
                          keying="pair"):
    """The library's pair records of outer point 4 n + k (rec from
    debug_pairs) against the oracle's brute force over every tet: the same
    inner tets and classes (asserted), and the moment error of moment_errors.
    Returns (error, near ties of the point)."""
    cls, S, ties = orc.point_moments(mesh.coords, mesh.tets, int(n), k, delta, N, seed, strategy=strategy,
                                     cap_sampling=cap_sampling, keying=keying, with_ties=True)
    sel = rec["q"] == 4 * int(n) + k
    mm = rec["m"][sel]
    order = np.argsort(mm)
    mm = mm[order]
    assert np.array_equal(mm, np.nonzero(cls)[0])
    assert np.array_equal(rec["cls"][sel][order], cls[mm])
    n_min = N // 3 if cap_sampling == "outside_ui" else N
    weight = tet_volumes(mesh.coords, mesh.tets[mm]) / max(n_min, 1)
    return moment_errors(rec["S"][sel][order], S[mm], ties[mm], weight), int(ties[mm].sum())
