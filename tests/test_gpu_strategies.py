"""Ball approximation strategies (Sec. 4.1: nocaps, overlap, inside,
barycenter beside fullcaps) on the GPU against the oracle: pair counts and
CSR pattern bit-exact, FP64 entries within 1e-12 of the row scale (and
1e-12 relative on entries above 1e-4 of it), on the plain workload and a
seeded subset of the precision workload; the strategy code is validated at
the boundary."""
import sys

import numpy as np
import pytest

import meshgen as mg
import helpers as H

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-6  # the form reaches about 1e-7 of the row scale on outer subsets (float subtet moments)
STRATS = ["nocaps", "overlap", "inside", "barycenter"]


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


def _check(dev, orc, pb, mask=None, tol=FP64_TOL):
    import paper_2302_07499_amd as P
    _say(f"{pb.name} strategy {pb.strategy} {pb.precision} K={pb.mesh.n_tets}")
    plan = dev.plan_problem(pb, outer_mask=mask)
    g = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal))
    o = orc.problem_assemble(pb, outer_mask=mask)
    assert np.array_equal(g["pair_counts"], o["pair_counts"]), (g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"  pairs {o['pair_counts']} errors {e}")
    assert e["ff_abs"] <= tol and e["fc_abs"] <= tol and e["rhs"] <= tol, e
    if tol == FP64_TOL:
        # relative bar on entries above 1e-4 of their row scale: smaller entries
        # are sums that cancel, whose relative error is not an FP64 property
        sc = H.row_scale(o)
        for blk in ["ff", "fc"]:
            rows = np.repeat(np.arange(o["n_free"]), np.diff(o[blk + "_row_ptr"]))
            a, b = np.asarray(g[blk + "_val"]), np.asarray(o[blk + "_val"])
            big = np.abs(b) > 1e-4 * sc[rows]
            if big.any():
                assert np.max(np.abs(a - b)[big] / np.abs(b)[big]) <= tol, blk
    plan.destroy()
    return g, o


@pytest.mark.parametrize("strategy", STRATS)
def test_plain_strategy(dev, orc, strategy):
    pb = mg.plain_problem()
    pb.strategy = strategy
    g, o = _check(dev, orc, pb)
    if strategy in ("overlap", "inside", "barycenter"):
        assert np.all(o["pair_counts"][1:] == 0)  # whole elements only


@pytest.mark.parametrize("strategy", ["nocaps", "barycenter"])
def test_precision_subset_strategy(dev, orc, strategy):
    pb = mg.precision_problem()
    pb.strategy = strategy
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 0.001, seed=21)
    _check(dev, orc, pb, mask)


def test_fp32_local_nocaps(dev, orc):
    pb = mg.make_problem("jit", 8, delta_over_h=3.0, jitter=0.2, jitter_seed=5, mc_samples=16, seed=2,
                         precision="fp32")
    pb.strategy = "nocaps"
    _check(dev, orc, pb, tol=FP32_TOL)


def test_unknown_strategy_rejected(dev):
    import paper_2302_07499_amd as P
    m = mg.kuhn_cube_mesh(2)
    vf = mg.free_mask_box(m.coords, 0.3)
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, 0.3, 1.0, 8, 0, strategy=5)
    assert ei.value.status == P.NLFEM_E_INVALID_ARG


# ---- cap sampling on E_m minus U_I (corner tet for n_in = 3, three cone tets for n_in = 1, 2)
def test_plain_region_cap_sampling(dev, orc):
    pb = mg.plain_problem()
    pb.cap_sampling = "outside_ui"
    _check(dev, orc, pb)


def test_precision_subset_region_cap_sampling(dev, orc):
    pb = mg.precision_problem()
    pb.cap_sampling = "outside_ui"
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 0.001, seed=23)
    _check(dev, orc, pb, mask)


def test_region_cap_sampling_pair_moments(dev, orc):
    """per-pair moments of every pair of two outer tets against the oracle,
    cut pairs of every n_in among them"""
    import paper_2302_07499_amd as P
    pb = mg.make_problem("jit", 8, delta_over_h=3.0, jitter=0.2, jitter_seed=5, mc_samples=32, seed=3)
    pb.cap_sampling = "outside_ui"
    plan = dev.plan_problem(pb)
    region = np.array([pb.vertex_free[t].any() for t in pb.mesh.tets])
    outer = np.nonzero(region)[0]
    seen = {3: 0, 4: 0, 5: 0}
    for n in outer[[0, len(outer) // 2]]:
        rec = plan.debug_pairs(4 * int(n), 4 * int(n) + 4)
        for k in range(4):
            err, t = H.point_pairs_vs_oracle(orc, pb.mesh, rec, n, k, pb.delta, pb.mc_samples, pb.seed,
                                             cap_sampling="outside_ui")
            assert err <= 1e-12, (n, k, err)
            cls = rec["cls"][rec["q"] == 4 * n + k]
            for c in (3, 4, 5):
                seen[c] += int((cls == c).sum())
    assert min(seen.values()) > 0, seen
    plan.destroy()


def test_region_cap_sampling_needs_three_samples(dev):
    import paper_2302_07499_amd as P
    m = mg.kuhn_cube_mesh(2)
    vf = mg.free_mask_box(m.coords, 0.3)
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, 0.3, 1.0, 2, 0, cap_sampling="outside_ui")
    assert ei.value.status == P.NLFEM_E_INVALID_ARG


def test_unknown_cap_sampling_rejected(dev):
    import paper_2302_07499_amd as P
    m = mg.kuhn_cube_mesh(2)
    vf = mg.free_mask_box(m.coords, 0.3)
    with pytest.raises(P.NlfemError) as ei:
        dev.plan(m.coords, m.tets, vf, 0.3, 1.0, 8, 0, cap_sampling=2)
    assert ei.value.status == P.NLFEM_E_INVALID_ARG
