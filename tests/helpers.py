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
    above 1e-6 of the row scale), rhs relative error."""
    sc = row_scale(o)
    out = {}
    for blk in ["ff", "fc"]:
        rp = o[blk + "_row_ptr"]
        rows = np.repeat(np.arange(o["n_free"]), np.diff(rp))
        a, b = np.asarray(g[blk + "_val"]), np.asarray(o[blk + "_val"])
        if len(b) == 0:
            out[blk + "_abs"] = 0.0
            out[blk + "_rel"] = 0.0
            continue
        d = np.abs(a - b)
        s = np.maximum(sc[rows], 1e-300)
        out[blk + "_abs"] = float(np.max(d / s))
        big = np.abs(b) > 1e-6 * s
        out[blk + "_rel"] = float(np.max(d[big] / np.abs(b[big]))) if big.any() else 0.0
    rb = np.asarray(o["rhs"])
    if len(rb):
        out["rhs"] = float(np.max(np.abs(np.asarray(g["rhs"]) - rb)) / max(np.max(np.abs(rb)), 1e-300))
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
