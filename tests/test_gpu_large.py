"""Large workload (64^3 Kuhn cubes, 1,572,864 tets, jitter 0.2h, delta = 4h,
N = 128, FP32-local): the full assembly in the benchmark's launch
configuration checked by properties that hold at any size (A 1 = 0,
symmetry on sampled rows, CG convergence) and by sampled outer points
against the oracle's brute force; plus a seeded subset of outer tets on the
full mesh against the oracle's assembly."""
import sys
import time

import numpy as np
import pytest

import meshgen as mg
import helpers as H

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-6  # the form reaches about 1e-7 of the row scale on outer subsets (float subtet moments)


def _say(msg):
    sys.stdout.write(f"[gpu-test] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_07499_amd as P
    d = P.Device(0)
    yield d
    d.close()


@pytest.fixture(scope="module")
def large():
    return mg.large_problem()


def test_large_full_properties_and_sampled_points(dev, orc, large):
    import paper_2302_07499_amd as P
    pb = large
    t0 = time.time()
    _say(f"large: plan + assemble, K={pb.mesh.n_tets} delta={pb.delta:.5g} N={pb.mc_samples} {pb.precision}")
    plan = dev.plan_problem(pb)
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    info = plan.info
    _say(f"large: assembled in {time.time() - t0:.1f} s, pairs {info['pair_counts']}, nnz_ff {info['nnz_ff']}, "
         f"nnz_fc {info['nnz_fc']}, timings {plan.timings()}")
    x, it, rr, ok = plan.solve(s, rtol=1e-10)
    _say(f"large: CG {it} iterations, rel residual {rr:.3e}")
    assert ok and rr <= 1e-10
    g = P.system_to_numpy(s)
    nf = g["n_free"]
    # A 1 = 0 per row (relative to the row's absolute sum)
    tot = np.zeros(nf)
    mag = np.zeros(nf)
    for blk in ["ff", "fc"]:
        rp, v = g[blk + "_row_ptr"], g[blk + "_val"]
        cnt = np.diff(rp)
        rows = np.repeat(np.arange(nf), cnt)
        tot += np.bincount(rows, weights=v, minlength=nf)
        mag += np.bincount(rows, weights=np.abs(v), minlength=nf)
    assert np.all(np.abs(tot) <= FP32_TOL * mag)
    # symmetry of A_ff on sampled rows
    rp, ci, va = g["ff_row_ptr"], g["ff_col"], g["ff_val"]
    rows = np.repeat(np.arange(nf, dtype=np.int64), np.diff(rp))
    keys = rows * nf + ci
    rng = np.random.default_rng(3)
    sample = rng.choice(nf, size=min(2000, nf), replace=False)
    sel = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in sample])
    tkeys = ci[sel].astype(np.int64) * nf + rows[sel]
    pos = np.searchsorted(keys, tkeys)
    assert np.all(keys[pos] == tkeys)
    scale = np.abs(va).max()
    assert np.max(np.abs(va[pos] - va[sel])) <= 1e-14 * scale
    _say("large: row sums and symmetry ok; sampled outer points vs oracle")
    m = pb.mesh
    region = np.array([pb.vertex_free[t].any() for t in m.tets])
    outer = np.nonzero(region)[0]
    for n in rng.choice(outer, size=2, replace=False):
        rec = plan.debug_pairs(4 * int(n), 4 * int(n) + 4)
        for k in range(4):
            err, t = H.point_pairs_vs_oracle(orc, m, rec, n, k, pb.delta, pb.mc_samples, pb.seed)
            assert err <= FP32_TOL, (n, k, err)
    plan.destroy()


def test_large_subset_vs_oracle(dev, orc, large):
    pb = large
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 1e-4, seed=17)
    _say(f"large subset: {int(mask.sum())} tets in the mask")
    plan = dev.plan_problem(pb, outer_mask=mask)
    import paper_2302_07499_amd as P
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    g = P.system_to_numpy(s)
    t0 = time.time()
    o = orc.problem_assemble(pb, outer_mask=mask)
    _say(f"large subset: oracle {time.time() - t0:.1f} s, pairs {o['pair_counts']}")
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"large subset fp32-local errors {e}")
    assert e["ff_abs"] <= FP32_TOL and e["fc_abs"] <= FP32_TOL and e["rhs"] <= FP32_TOL
    plan.destroy()
