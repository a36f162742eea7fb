"""Serving: requests of mixed sizes, horizons, sample counts and precisions run
through the request server.  Each solution is the same alone and in the mix
(bitwise), matches the single-plan path and the oracle, and admission keeps
the running requests inside the memory pool."""
import sys

import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

WAIT_S = 120.0


def _say(msg):
    sys.stdout.write(f"[gpu-test] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_07499_amd as P
    return P


def _requests(count=8, seed=31):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(rng.integers(4, 11))
        out.append(mg.make_problem(f"req{r}", n, delta_over_h=float(rng.uniform(2.0, 3.5)), jitter=0.15,
                                   jitter_seed=700 + r, mc_samples=int(rng.choice([8, 16, 32])), seed=r,
                                   precision=str(rng.choice(["fp64", "fp32"]))))
    # a request with no free vertex (n = 6, delta = 3h) in the mix
    out.append(mg.make_problem("empty", 6, delta_over_h=3.0, jitter=0.15, jitter_seed=9, mc_samples=8))
    return out


def _run_alone(P, pbs):
    sv = P.Server(0, n_slots=1, pool_bytes=4 << 30)
    xs = []
    for pb in pbs:
        t = sv.submit(pb)
        info = sv.wait(t, WAIT_S)
        assert info["state"] == 2, info
        x, f2v, _ = sv.take(t)
        xs.append((x, f2v))
    sv.close()
    return xs


def test_alone_equals_mix_and_single_plan(gpu):
    P = gpu
    pbs = _requests()
    alone = _run_alone(P, pbs)
    sv = P.Server(0, n_slots=4, pool_bytes=4 << 30)
    tickets = [sv.submit(pb) for pb in pbs]
    infos = [sv.wait(t, WAIT_S) for t in tickets]
    mix = [sv.take(t)[:2] for t in tickets]
    st = sv.stats()
    sv.close()
    _say(f"mix stats {st}")
    assert st["done"] == len(pbs) and st["failed"] == 0
    assert st["max_running"] >= 2
    for i, (a, m) in enumerate(zip(alone, mix)):
        assert infos[i]["state"] == 2 and infos[i]["status"] == 0, infos[i]
        assert np.array_equal(a[0], m[0]), i
        assert np.array_equal(a[1], m[1]), i
    # the single-plan path on the device context's stream gives the same solution
    dev = P.Device(0)
    for i, pb in enumerate(pbs):
        plan = dev.plan_problem(pb)
        s = plan.assemble(pb.f_qp, pb.g_nodal)
        x, it, rr, ok = plan.solve(s, rtol=1e-10)
        assert np.array_equal(x.cpu().numpy(), alone[i][0]), i
        plan.destroy()
    dev.close()


def test_served_solution_matches_oracle(gpu, orc):
    P = gpu
    pb = mg.plain_problem()
    sv = P.Server(0, n_slots=2, pool_bytes=1 << 30)
    t = sv.submit(pb)
    info = sv.wait(t, WAIT_S)
    x, f2v, _ = sv.take(t)
    sv.close()
    assert info["state"] == 2 and info["cg_rel_residual"] <= 1e-10
    o = orc.problem_assemble(pb)
    xo, ito, rro, rc = orc.cg(o["ff_row_ptr"], o["ff_col"], o["ff_val"], o["rhs"], rtol=1e-10)
    assert np.array_equal(f2v, np.flatnonzero(pb.vertex_free))
    assert abs(info["cg_iters"] - ito) <= 1
    assert np.max(np.abs(x - xo)) <= 1e-9 * np.max(np.abs(xo))


def test_admission_by_footprint_and_oversized_request(gpu):
    P = gpu
    pbs = _requests(6, seed=5)
    alone = _run_alone(P, pbs)
    pool = 256 << 20
    sv = P.Server(0, n_slots=4, pool_bytes=pool)
    tickets = [sv.submit(pb) for pb in pbs]
    # far larger than the pool: must fail with E_OOM after running alone, without hurting the others
    big = mg.make_problem("big", 20, delta_over_h=4.0, jitter=0.15, jitter_seed=3, mc_samples=8)
    tb = sv.submit(big)
    infos = [sv.wait(t, WAIT_S) for t in tickets]
    ib = sv.wait(tb, WAIT_S)
    st = sv.stats()
    _say(f"small pool stats {st}; estimates {[i['est_bytes'] >> 20 for i in infos]} MiB, "
         f"peaks {[i['peak_bytes'] >> 20 for i in infos]} MiB; big {ib}")
    for i, t in enumerate(tickets):
        assert infos[i]["state"] == 2, infos[i]
        x, f2v, _ = sv.take(t)
        assert np.array_equal(x, alone[i][0]), i
    assert ib["state"] == 3 and ib["status"] == P.NLFEM_E_OOM
    assert st["pool_peak"] <= pool
    # admission keeps the sum of estimates inside the pool
    est_min = min(i["est_bytes"] for i in infos)
    assert st["max_running"] <= max(1, pool // est_min)
    sv.close()


def test_poisson_stream_latency(gpu):
    P = gpu
    import time
    rng = np.random.default_rng(8)
    pbs = _requests(16, seed=77)
    gaps = rng.exponential(0.01, size=len(pbs))
    sv = P.Server(0, n_slots=4, pool_bytes=4 << 30)
    tickets = []
    for pb, gap in zip(pbs, gaps):
        time.sleep(float(gap))
        tickets.append(sv.submit(pb))
    infos = [sv.wait(t, WAIT_S) for t in tickets]
    lat = np.array([i["latency_s"] for i in infos])
    st = sv.stats()
    sv.close()
    assert all(i["state"] == 2 for i in infos)
    for i in infos:
        assert i["latency_s"] >= i["queue_s"] + i["plan_s"] + i["assemble_s"] + i["solve_s"] - 1e-6
    _say(f"stream of {len(pbs)}: p50 {np.percentile(lat, 50) * 1e3:.1f} ms p99 {np.percentile(lat, 99) * 1e3:.1f} ms, "
         f"max running {st['max_running']}")
