"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: classification, pair lists and CSR pattern bit-exact; FP64 entries
within 1e-12 of the row scale (and 1e-12 relative on entries above 1e-6 of
it); FP32-local entries within 1e-6 of the row scale; CG solutions within
1e-9 relative.
"""
import os
import sys

import numpy as np
import pytest

import meshgen as mg
import helpers as H

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
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


def _gpu_system(dev, pb, outer_mask=None, precision=None):
    import paper_2302_07499_amd as P
    if precision is not None:
        pb.precision = precision
    _say(f"plan {pb.name} n={pb.mesh.n} K={pb.mesh.n_tets} delta={pb.delta:.5g} N={pb.mc_samples} {pb.precision}")
    plan = dev.plan_problem(pb, outer_mask=outer_mask)
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    return plan, s, P.system_to_numpy(s)


@pytest.fixture(scope="module")
def plain(dev, orc):
    pb = mg.plain_problem()
    plan, s, g = _gpu_system(dev, pb)
    o = orc.problem_assemble(pb)
    return pb, plan, s, g, o


def test_plain_pattern_and_pair_counts(plain):
    pb, plan, s, g, o = plain
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)


def test_plain_values_fp64(plain):
    pb, plan, s, g, o = plain
    e = H.value_errors(g, o)
    _say(f"plain fp64 errors {e}")
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL
    assert e["ff_rel"] <= FP64_TOL and e["fc_rel"] <= FP64_TOL
    assert e["rhs"] <= FP64_TOL


def test_plain_pair_moments_match_oracle(plain, orc):
    """Every non-OUT pair of a few outer points: same class, moments equal to
    1e-14 relative (same samples; Monte Carlo sums are exact dyadics)."""
    pb, plan, s, g, o = plain
    m = pb.mesh
    region = np.array([pb.vertex_free[t].any() for t in m.tets])
    outer = np.nonzero(region)[0]
    ties = 0
    for n in outer[:: max(1, len(outer) // 6)]:
        rec = plan.debug_pairs(4 * int(n), 4 * int(n) + 4)
        for k in range(4):
            err, t = H.point_pairs_vs_oracle(orc, m, rec, n, k, pb.delta, pb.mc_samples, pb.seed)
            ties += t
            assert err <= 1e-14, (n, k, err)
    _say(f"plain pair moments: near ties of the sample test {ties}")


def test_plain_invariants_and_determinism(dev, plain):
    import paper_2302_07499_amd as P
    pb, plan, s, g, o = plain
    tot, mag = H.row_sums(g)
    assert np.all(np.abs(tot) <= 1e-12 * mag)
    A = H.dense_ff(g)
    assert np.max(np.abs(A - A.T)) <= 1e-14 * np.abs(A).max()
    s2 = plan.assemble(pb.f_qp, pb.g_nodal)
    g2 = P.system_to_numpy(s2)
    for k in ["ff_val", "fc_val", "rhs"]:
        assert np.array_equal(g[k], g2[k]), k


def test_plain_cg_matches_oracle(plain, orc):
    pb, plan, s, g, o = plain
    x, it, rr, ok = plan.solve(s, rtol=1e-10)
    assert ok and rr <= 1e-10
    xo, ito, rro, rc = orc.cg(o["ff_row_ptr"], o["ff_col"], o["ff_val"], o["rhs"], rtol=1e-10)
    xg = x.cpu().numpy()
    assert abs(it - ito) <= 1
    assert np.max(np.abs(xg - xo)) <= 1e-9 * np.max(np.abs(xo))


def test_plain_cg_device_poll_and_plan_form(dev, plain):
    """The device-side stopping decision gives the same iterations and the
    same bits through the raw-CSR and the plan entry points; a capped solve
    reports its exact iteration count."""
    import paper_2302_07499_amd as P
    pb, plan, s, g, o = plain
    x, it, rr, ok = plan.solve(s, rtol=1e-10)
    t = dev.torch
    x2 = t.zeros(s.n_free, dtype=t.float64, device=dev.dev)
    it2, rr2, ok2 = P.nlfem_plan_cg(plan.handle, s.n_free, s.ff_val, s.rhs, x2, rtol=1e-10, ctx=dev.ctx)
    assert ok and ok2 and it2 == it and rr2 == rr
    assert t.equal(x, x2)
    for cap in (1, 3, it - 1):
        x3 = t.zeros(s.n_free, dtype=t.float64, device=dev.dev)
        it3, rr3, ok3 = P.nlfem_cg(dev.ctx, s.n_free, s.ff_row_ptr, s.ff_col, s.ff_val, s.rhs, x3, 1e-10, cap)
        assert not ok3 and it3 == cap and rr3 > 1e-10


def test_row_buffer_overflow_retry(dev, plain):
    """A row buffer far too narrow for the CSR rows (16 words a row, set by
    NLFEM_ROW_STRIDE) makes the count pass report the overflow and run again
    with wider strides; the pattern and values are bitwise those of the
    plain plan."""
    pb, plan, s, g, o = plain
    os.environ["NLFEM_ROW_STRIDE"] = "16"
    try:
        plan2, s2, g2 = _gpu_system(dev, mg.plain_problem())
    finally:
        del os.environ["NLFEM_ROW_STRIDE"]
    for k in ["ff_row_ptr", "ff_col", "fc_row_ptr", "fc_col", "ff_val", "fc_val", "rhs"]:
        assert np.array_equal(g[k], g2[k]), k
    plan2.destroy()


def test_local_vertex_set_handoff_fallback(dev, plain):
    """Local vertex sets longer than the count pass's hand-off buffer (16
    entries a set, set by NLFEM_VE_STRIDE) are built again by the fill pass;
    the plain plan takes the hand-off; pattern and values bitwise equal."""
    pb, plan, s, g, o = plain
    os.environ["NLFEM_VE_STRIDE"] = "16"
    try:
        plan2, s2, g2 = _gpu_system(dev, mg.plain_problem())
    finally:
        del os.environ["NLFEM_VE_STRIDE"]
    for k in ["ff_row_ptr", "ff_col", "fc_row_ptr", "fc_col", "ff_val", "fc_val", "rhs"]:
        assert np.array_equal(g[k], g2[k]), k
    plan2.destroy()


def test_cg_breakdown_on_indefinite_matrix(dev):
    """An indefinite matrix makes p.Ap <= 0: the solve stops at once with
    NLFEM_E_NOT_CONVERGED and a breakdown message instead of running to the cap."""
    import paper_2302_07499_amd as P
    t = dev.torch
    n = 64
    rp = t.arange(n + 1, dtype=t.int64, device=dev.dev)
    ci = t.arange(n, dtype=t.int32, device=dev.dev)
    va = t.ones(n, dtype=t.float64, device=dev.dev)
    va[1::2] = -1.0
    b = t.zeros(n, dtype=t.float64, device=dev.dev)
    b[0], b[1] = 1.0, 1.0
    x = t.zeros(n, dtype=t.float64, device=dev.dev)
    it, rr, ok = P.nlfem_cg(dev.ctx, n, rp, ci, va, b, x, 1e-10, 1000)
    assert not ok and it == 1
    assert "breakdown" in P.last_error(dev.ctx)
    # b = 0: x = 0 at once
    x.fill_(5.0)
    it, rr, ok = P.nlfem_cg(dev.ctx, n, rp, ci, t.ones(n, dtype=t.float64, device=dev.dev), t.zeros_like(b), x,
                            1e-10, 10)
    assert ok and it == 0 and float(x.abs().max()) == 0.0


def test_plain_fp32_local(dev, plain):
    pb, plan, s, g, o = plain
    pb32 = mg.plain_problem()
    plan32, s32, g32 = _gpu_system(dev, pb32, precision="fp32")
    H.pattern_equal(g32, o)
    e = H.value_errors(g32, o)
    _say(f"plain fp32-local errors {e}")
    assert e["ff_abs"] <= FP32_TOL and e["fc_abs"] <= FP32_TOL and e["rhs"] <= FP32_TOL


@pytest.fixture(scope="module")
def precision_subset(dev, orc):
    """Precision workload (32^3 cubes, jitter 0.2h, delta = 3h, N = 64) on a
    deterministic subset of about 0.15% of the outer tets."""
    pb = mg.precision_problem()
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 0.0015, seed=11)
    plan, s, g = _gpu_system(dev, pb, outer_mask=mask)
    _say("oracle on the subset ...")
    o = orc.problem_assemble(pb, outer_mask=mask)
    return pb, mask, plan, s, g, o


def test_precision_subset_fp64(precision_subset):
    pb, mask, plan, s, g, o = precision_subset
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"precision subset fp64 errors {e}")
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL
    assert e["ff_rel"] <= FP64_TOL and e["fc_rel"] <= FP64_TOL
    assert e["rhs"] <= FP64_TOL


def test_precision_subset_fp32(dev, precision_subset):
    pb, mask, plan, s, g, o = precision_subset
    pb32 = mg.precision_problem("fp32")
    plan32, s32, g32 = _gpu_system(dev, pb32, outer_mask=mask)
    H.pattern_equal(g32, o)
    e = H.value_errors(g32, o)
    _say(f"precision subset fp32-local errors {e}")
    assert e["ff_abs"] <= FP32_TOL and e["fc_abs"] <= FP32_TOL and e["rhs"] <= FP32_TOL


def _slab_problem(n, delta_over_h):
    """n x n Kuhn cubes one cube thick in x (the first layer of the n^3 cube
    mesh, vertices renumbered), free where min(y, 1-y, z, 1-z) > delta."""
    full = mg.kuhn_cube_mesh(n)
    keep = (np.arange(full.n_tets) // 6) % n == 0
    T = full.tets[keep]
    used = np.unique(T)
    remap = np.full(full.coords.shape[0], -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    X = np.ascontiguousarray(full.coords[used])
    mesh = mg.Mesh(coords=X, tets=np.ascontiguousarray(remap[T].astype(np.int32)), n=n, h=1.0 / n,
                   info={"kind": "slab"})
    delta = delta_over_h / n
    yz = X[:, 1:]
    free = (np.minimum(yz, 1.0 - yz).min(axis=1) > delta).astype(np.uint8)
    return mg.Problem(name="slab", mesh=mesh, delta=delta, psi=mg.psi_unit_laplacian(delta), mc_samples=8,
                      seed=4, vertex_free=free, f_qp=mg.const_f_qp(mesh.n_tets, -2.0),
                      g_nodal=mg.g_x1_squared(X))


def test_wide_horizon_candidate_rows(dev, orc):
    """A 32 x 32 slab of cubes one cube thick with delta = 10h: the ball of an
    outer tet spans 484 to 625 cell rows of the candidate grid, more than the
    fast classification keeps in LDS at a time (256), so it walks them in
    batches; the ball meets only the slab, so the vertex sets still fit."""
    pb = _slab_problem(32, 10.0)
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 0.1, seed=12)
    plan, s, g = _gpu_system(dev, pb, outer_mask=mask)
    o = orc.problem_assemble(pb, outer_mask=mask)
    plan.destroy()
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"slab fp64 errors {e}")
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL
    assert e["ff_rel"] <= FP64_TOL and e["fc_rel"] <= FP64_TOL
    assert e["rhs"] <= FP64_TOL


def test_precision_full_sampled_points(dev, orc):
    """Full precision workload in the benchmark's configuration: pair lists and
    moments of sampled outer points against the oracle's brute force, plus
    A 1 = 0 and symmetry over the whole matrix."""
    import paper_2302_07499_amd as P
    pb = mg.precision_problem()
    plan, s, g = _gpu_system(dev, pb)
    tot, mag = H.row_sums(g)
    assert np.all(np.abs(tot) <= 1e-12 * mag)
    A = H.sparse_ff(g)
    d = abs(A - A.T)
    assert d.max() <= 1e-14 * abs(A).max()
    m = pb.mesh
    region = np.array([pb.vertex_free[t].any() for t in m.tets])
    outer = np.nonzero(region)[0]
    rng = np.random.default_rng(5)
    ties = 0
    for n in rng.choice(outer, size=3, replace=False):
        rec = plan.debug_pairs(4 * int(n), 4 * int(n) + 4)
        for k in range(4):
            err, t = H.point_pairs_vs_oracle(orc, m, rec, n, k, pb.delta, pb.mc_samples, pb.seed)
            ties += t
            assert err <= 1e-14, (n, k, err)
    _say(f"precision full-size sampled points: near ties of the sample test {ties}")


# ---------------------------------------------------------------- edge cases --
def test_empty_system(dev, orc):
    """n = 8, delta/h = 4: no free vertex -> empty system, CG returns at once."""
    pb = mg.make_problem("empty", 8, delta_over_h=4.0, jitter=0.15, jitter_seed=3, mc_samples=8)
    assert pb.vertex_free.sum() == 0
    plan, s, g = _gpu_system(dev, pb)
    assert g["n_free"] == 0 and plan.info["nnz_ff"] == 0
    x, it, rr, ok = plan.solve(s)
    assert ok and it == 0


def test_single_tet_and_tiny_meshes(dev, orc):
    import paper_2302_07499_amd as P
    m = mg.six_tet_cube_mesh()
    vf = np.ones(m.n_vertices, np.uint8)
    for delta, N in [(0.3, 16), (0.5, 33), (0.8, 7)]:
        plan = dev.plan(m.coords, m.tets, vf, delta, 1.3, N, 4)
        g = P.system_to_numpy(plan.assemble(np.ones((6, 4)), None))
        o = orc.assemble(m.coords, m.tets, vf, delta, 1.3, N, 4, f_qp=np.ones((6, 4)))
        H.pattern_equal(g, o)
        e = H.value_errors(g, o)
        assert e["ff_abs"] <= FP64_TOL and e["rhs"] <= FP64_TOL, (delta, e)
    t = mg.single_tet_mesh(0.5)
    vf = np.array([1, 0, 0, 0], np.uint8)
    plan = dev.plan(t.coords, t.tets, vf, 0.2, 2.0, 12, 1)
    g = P.system_to_numpy(plan.assemble(None, np.arange(4.0)))
    o = orc.assemble(t.coords, t.tets, vf, 0.2, 2.0, 12, 1, g_nodal=np.arange(4.0))
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL and e["rhs"] <= FP64_TOL


def test_error_paths(dev, orc):
    import paper_2302_07499_amd as P
    m = mg.kuhn_cube_mesh(2)
    vf = mg.free_mask_box(m.coords, 0.3)
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, -1.0, 1.0, 8, 0)
    assert ei.value.status == P.NLFEM_E_INVALID_ARG
    bad = m.tets.copy()
    bad[3, 2] = m.n_vertices + 5
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, bad, vf, 0.3, 1.0, 8, 0)
    assert ei.value.status == P.NLFEM_E_MESH
    flat = m.coords.copy()
    flat[m.tets[0]] = flat[m.tets[0][0]]
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(flat, m.tets, vf, 0.3, 1.0, 8, 0)
    assert ei.value.status == P.NLFEM_E_MESH
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, 0.3, 1.0, 0, 0)
    assert ei.value.status == P.NLFEM_E_INVALID_ARG
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, 0.3, 1.0, P.NLFEM_MAX_MC_SAMPLES + 1, 0)
    assert ei.value.status == P.NLFEM_E_INVALID_ARG
    # the largest sample count is accepted and its sums stay exact: the oracle agrees
    pb = mg.make_problem("maxn", 4, delta_over_h=1.5, jitter=0.1, jitter_seed=2,
                         mc_samples=P.NLFEM_MAX_MC_SAMPLES, seed=4)
    plan = dev.plan_problem(pb)
    g = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal))
    o = orc.problem_assemble(pb)
    e = H.value_errors(g, o)
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL and e["rhs"] <= FP64_TOL, e
    plan.destroy()
    tiny = P.Device(0, hbm_budget_bytes=4096)
    with pytest.raises(P.NlfemError) as ei:
        tiny.plan(m.coords, m.tets, vf, 0.3, 1.0, 8, 0)
    assert ei.value.status == P.NLFEM_E_OOM
    tiny.close()
