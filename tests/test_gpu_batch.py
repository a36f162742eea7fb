"""Batched assembly (integration launches grouped by LDS footprint, replayed from a HIP graph):
each mesh's result equals its single-mesh assembly bitwise, on every graph
replay, and matches the oracle."""
import sys

import numpy as np
import pytest

import helpers as H
import meshgen as mg

FP32_TOL = 1e-6  # the form reaches about 1e-7 of the row scale on outer subsets (float subtet moments)

pytestmark = pytest.mark.gpu


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


def _mix(precision, count=10, seed=21):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(4, 10))
        r = float(rng.choice([2.0, 3.0, 4.0]))
        out.append(mg.make_problem(f"mix{b}", n, delta_over_h=r, jitter=0.15, jitter_seed=500 + b,
                                   mc_samples=int(rng.choice([8, 16, 33])), seed=b, precision=precision))
    # one mesh with no free vertex (n = 8, delta = 4h) in the mix
    out.append(mg.make_problem("empty", 8, delta_over_h=4.0, jitter=0.15, jitter_seed=3, mc_samples=8,
                               precision=precision))
    return out


def _eager(dev, pb):
    import paper_2302_07499_amd as P
    plan = dev.plan_problem(pb)
    s = plan.assemble(pb.f_qp, pb.g_nodal)
    g = P.system_to_numpy(s)
    plan.destroy()
    return g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_and_replays(dev, precision):
    import torch
    import paper_2302_07499_amd as P
    pbs = _mix(precision)
    _say(f"batch of {len(pbs)} meshes, {precision}")
    batch = P.Batch(dev, pbs)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    single = [_eager(dev, pb) for pb in pbs]
    for rep in range(3):
        batch.assemble()
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (x * 2.0).sum().item()
        for i, pb in enumerate(pbs):
            g = batch.system_numpy(i)
            H.pattern_equal(g, single[i])
            for k in ["ff_val", "fc_val", "rhs"]:
                assert np.array_equal(g[k], single[i][k]), (rep, i, k)
    _say(f"tuning {batch.tuning()}")
    batch.destroy()


def test_batch_lds_groups(dev):
    """Meshes whose local vertex sets need different LDS footprints (delta = 2h
    on small meshes, delta = 4h on a larger one) run as separate launches of
    one graph; each result equals its single-mesh assembly bitwise."""
    import paper_2302_07499_amd as P
    pbs = [mg.make_problem("g2a", 6, delta_over_h=2.0, jitter=0.15, jitter_seed=31, mc_samples=16, seed=1),
           mg.make_problem("g4", 14, delta_over_h=4.0, jitter=0.15, jitter_seed=32, mc_samples=16, seed=2),
           mg.make_problem("g2b", 9, delta_over_h=2.0, jitter=0.15, jitter_seed=33, mc_samples=16, seed=3)]
    batch = P.Batch(dev, pbs)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    batch.assemble()
    for i, pb in enumerate(pbs):
        g = batch.system_numpy(i)
        e = _eager(dev, pb)
        for k in ["ff_val", "fc_val", "rhs"]:
            assert np.array_equal(g[k], e[k]), (i, k)
    _say(f"lds groups: tuning {batch.tuning()}")
    batch.destroy()


@pytest.mark.parametrize("shape", [(256, 3), (128, 6), (256, 0), (128, 0)])
def test_batch_launch_shapes(dev, shape):
    """Both launch forms (persistent grid, one workgroup per item) and both
    workgroup sizes give each mesh's single-mesh result bitwise."""
    import paper_2302_07499_amd as P
    pbs = _mix("fp64", count=5, seed=9)
    batch = P.Batch(dev, pbs)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    batch.set_launch(*shape)
    batch.assemble()
    for i, pb in enumerate(pbs):
        g = batch.system_numpy(i)
        e = _eager(dev, pb)
        for k in ["ff_val", "fc_val", "rhs"]:
            assert np.array_equal(g[k], e[k]), (shape, i, k)
    _say(f"shape {shape}: tuning {batch.tuning()}")
    with pytest.raises(P.NlfemError):
        batch.set_launch(256, 4)  # 16 waves per CU
    batch.destroy()


def test_batch_matches_oracle(dev, orc):
    import paper_2302_07499_amd as P
    pbs = _mix("fp64", count=4, seed=5)
    batch = P.Batch(dev, pbs)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    batch.assemble()
    for i, pb in enumerate(pbs):
        g = batch.system_numpy(i)
        o = orc.problem_assemble(pb)
        assert np.array_equal(g["pair_counts"], o["pair_counts"])
        H.pattern_equal(g, o)
        e = H.value_errors(g, o)
        assert e["ff_abs"] <= 1e-12 and e["fc_abs"] <= 1e-12 and e["rhs"] <= 1e-12, (i, e)
    batch.destroy()


def test_batched_workload_subset_vs_oracle(dev, orc):
    """The 256-mesh batched workload's first 4 meshes (n up to 24, delta/h in
    {2,3,4}, jitter 0.15h, N = 32, FP32-local) on 1% outer-tet subsets."""
    import paper_2302_07499_amd as P
    pbs = mg.batched_problems(256)[:4]
    masks = [mg.outer_subset_mask(pb.mesh.n_tets, 0.01, seed=40 + i) for i, pb in enumerate(pbs)]
    batch = P.Batch(dev, pbs, outer_masks=masks)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    batch.assemble()
    for i, pb in enumerate(pbs):
        g = batch.system_numpy(i)
        o = orc.problem_assemble(pb, outer_mask=masks[i])
        assert np.array_equal(g["pair_counts"], o["pair_counts"])
        H.pattern_equal(g, o)
        e = H.value_errors(g, o)
        _say(f"batched mesh {i} n={pb.mesh.n} d/h={pb.info['delta_over_h']:.0f} fp32-local errors {e}")
        assert e["ff_abs"] <= FP32_TOL and e["fc_abs"] <= FP32_TOL and e["rhs"] <= FP32_TOL, (i, e)
    batch.destroy()


def test_batch_parallel_build_error_and_recovery(dev):
    """A batch of nine or more meshes builds its plans on several threads; a
    mesh with an out-of-range vertex index fails the whole batch with
    NLFEM_E_MESH (the plans already built are freed), and the context then
    builds a good batch whose results equal the single-mesh assemblies."""
    import dataclasses
    import paper_2302_07499_amd as P
    pbs = _mix("fp64", count=9, seed=13)
    bad_tets = pbs[5].mesh.tets.copy()
    bad_tets[2, 1] = pbs[5].mesh.n_vertices + 3
    bad = dataclasses.replace(pbs[5], mesh=dataclasses.replace(pbs[5].mesh, tets=bad_tets))
    before = P.nlfem_memory_in_use(dev.ctx)
    with pytest.raises(P.NlfemError) as ei:
        P.Batch(dev, pbs[:5] + [bad] + pbs[6:])
    assert ei.value.status == P.NLFEM_E_MESH
    assert P.nlfem_memory_in_use(dev.ctx) <= before + (64 << 20)
    _say("parallel build error reported; building the good batch")
    batch = P.Batch(dev, pbs)
    batch.set_inputs([pb.f_qp for pb in pbs], [pb.g_nodal for pb in pbs])
    batch.assemble()
    for i, pb in enumerate(pbs):
        g = batch.system_numpy(i)
        e = _eager(dev, pb)
        for k in ["ff_val", "fc_val", "rhs"]:
            assert np.array_equal(g[k], e[k]), (i, k)
    batch.destroy()
