#!/usr/bin/env python3
"""Benchmark: assembled (point, element) pairs per second of the fullcaps
assembly on one MI355X, FP64 and FP32-local, with the batched and served
forms beside it.

Main workload (the JSON line's value): 32^3 Kuhn-split cubes of [0,1]^3
(196,608 tets, 35,937 vertices), interior vertices jittered uniformly by
+-0.2h (seed 1), delta = 3h, psi = 15/(4 pi delta^5), N = 64 Monte Carlo
samples per cut pair, f = -2, g = x1^2.  One step is one pass of the whole
assembly path on the device: mesh layout, cell list, exact classification,
local vertex sets, row lists and CSR pattern (plan_create), then pair
integration, inner-element terms, row assembly and the right-hand side
(assemble).  Inputs are resident in HBM when the timed region starts; the CG
solve is timed separately.

Batched: 256 meshes (n ~ U{8..24}, delta/h in {2,3,4}, jitter 0.15h, N = 32,
FP32-local), one integration launch per LDS-footprint group of meshes per graph replay.

Strategies: the same workload assembled with the other ball approximations
(nocaps, overlap, inside, barycenter; FP64), one line each beside the main
fullcaps value, and fullcaps with the caps sampled on E - U_I (the corner tet
for n_in = 3, three cone tets for n_in = 1, 2), with the seed-to-seed spread of
the matrix entries in both modes.

Convergence: the paper's 3D accuracy experiment (Sec. 5) on synthetic meshes:
Omega = (0,1)^3, delta = 0.1, u = prod x_d (1 - x_d), Kuhn meshes h = 1/m
(m = 16..40) with a collar of whole cubes, N = 64, FP64; per strategy and level
the assembly time, CG iterations, L2 error, observed order and the paper's
efficiency ratio lambda.

Element keying: the main workload with N samples per element shared by the
outer points of an outer tet (FP64 and FP32-local), with the integration
kernel's roofline fraction.

Large: 64^3 Kuhn cubes (1,572,864 tets), jitter 0.2h, delta = 4h, N = 128,
FP64 and FP32-local: pairs/s, phase times, roofline fraction, CG.

Serving: a stream of 500 requests (n ~ U{8..40}, delta/h ~ U[2,5], N in
{32,64}, FP64 / FP32-local 50/50) through the request server: saturation
throughput with all requests queued at once, then Poisson streams at 0.5x
and 0.9x that rate for the latency percentiles (arrival -> solution in host
memory).

CPU baseline: the oracle (serial FP64 brute force) on a seeded 0.2 % subset of
the main workload's outer tets, with the host CPU model; the library's FP64,
FP32-local and element-keyed results on the same subset against it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X vector FP64: 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
# algorithmic FLOPs of the integration kernel (per unit; see the design notes)
FLOP_PER_SAMPLE = 56
FLOP_PER_CUT_PAIR = 700
FLOP_PER_IN_PAIR = 100


# HBM traffic of the integration kernel comes from rocprofv3 FETCH_SIZE /
# WRITE_SIZE counter runs summarised in this file; it is reported only while
# the kernel's sources and build flags hash to the digest recorded there.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_integrate_traffic_precision.txt")
# VALU instruction counters of the same kernel (rocprofv3 --pmc SQ_INSTS_VALU ...), same rule
VALU_RECORD = os.path.join(ROOT, "profiles", "k_integrate_valu_precision.txt")
INTEGRATE_SOURCES = ["paper_2302_07499_amd/csrc/k_numeric.hip", "paper_2302_07499_amd/csrc/device_geom.hpp",
                     "paper_2302_07499_amd/csrc/common.hpp", "paper_2302_07499_amd/build.py"]


def integrate_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in INTEGRATE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def _read_record(path):
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    return rec


def recorded_valu():
    """VALU issue figures of the integration kernel from the counter summary,
    or None when the kernel sources changed since."""
    try:
        rec = _read_record(VALU_RECORD)
        if rec.get("sources_sha256") != integrate_sources_digest():
            return None
        return {"issue_frac": float(rec["valu_issue_frac"]), "insts_per_launch": float(rec["valu_insts_per_launch"]),
                "hw_f64_flop_per_launch": float(rec["valu_f64_flop_per_launch"])}
    except (OSError, KeyError, ValueError):
        return None


def recorded_traffic():
    """(bytes per launch, record) from the counter summary, or (None, reason)."""
    try:
        rec = {}
        with open(TRAFFIC_RECORD) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip()
        if rec.get("sources_sha256") != integrate_sources_digest():
            return None, "kernel sources changed since the counters were taken"
        copy = float(rec["calibration_bytes"])
        fetch = float(rec["fetch_kib_per_launch"]) * copy / float(rec["copy_fetch_kib"])
        write = float(rec["write_kib_per_launch"]) * copy / float(rec["copy_write_kib"])
        return int(round(fetch + write)), {"fetch_bytes": int(round(fetch)), "write_bytes": int(round(write))}
    except (OSError, KeyError, ValueError) as e:
        return None, f"no usable counter record ({e.__class__.__name__})"


def host_cpu():
    """Model and logical CPU count of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def pct(a, q):
    return round(float(np.percentile(np.asarray(a), q)), 3) if len(a) else None


def flops_of(info, N):
    """Algorithmic FLOPs of one integration launch (per-unit model above)."""
    cut = int(sum(info["pair_counts"][1:]))
    inn = int(info["pair_counts"][0])
    return FLOP_PER_SAMPLE * cut * N + FLOP_PER_CUT_PAIR * cut + FLOP_PER_IN_PAIR * inn


class Stepper:
    """One workload resident in HBM; a step is plan_create + assemble on it
    (the whole assembly path), timed with a synchronised wall clock, with the
    library's HIP-event phase timings beside it."""

    def __init__(self, P, dev, pb, label):
        import torch
        self.P, self.dev, self.pb, self.label, self.torch = P, dev, pb, label, torch
        mesh = pb.mesh
        t = torch
        self.keep = [dev.to_dev(mesh.coords, t.float64), dev.to_dev(mesh.tets, t.int32),
                     dev.to_dev(pb.vertex_free, t.uint8)]
        self.d_f = dev.to_dev(pb.f_qp, t.float64)
        self.d_g = dev.to_dev(pb.g_nodal, t.float64)
        self.m = P.nlfem_mesh(mesh.n_vertices, mesh.n_tets, self.keep[0].data_ptr(), self.keep[1].data_ptr(),
                              self.keep[2].data_ptr(), None, 1)

    def params(self, precision, strategy="fullcaps", cap_sampling="whole", seed=None, keying="pair", mask=None):
        P, pb = self.P, self.pb
        return P.nlfem_params(pb.delta, pb.psi, pb.mc_samples, pb.seed if seed is None else seed,
                              P.NLFEM_FP32_LOCAL if precision == "fp32" else P.NLFEM_FP64,
                              None if mask is None else mask.data_ptr(), P.strategy_id(strategy),
                              P.cap_sampling_id(cap_sampling), P.keying_id(keying))

    def run(self, precision, steps, warmup, keep_last=True, **kw):
        P, dev, torch = self.P, self.dev, self.torch
        prm = self.params(precision, **kw)
        # allocate outputs once (sizes are the same every step)
        plan = P.Plan(dev, P.nlfem_plan_create(dev.ctx, self.m, prm))
        sysm = plan.alloc_system()
        plan.destroy()
        times, tk = [], []
        info = None
        last = None
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = P.nlfem_plan_create(dev.ctx, self.m, prm)
            P.nlfem_assemble(h, self.d_f, self.d_g, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val, sysm.fc_row_ptr,
                             sysm.fc_col, sysm.fc_val, sysm.rhs, sysm.free_to_vertex, ctx=dev.ctx)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if i >= warmup:
                times.append(t1 - t0)
                tk.append(P.nlfem_plan_timings(h))
            if info is None:
                info = P.nlfem_plan_info(h)
            if i == warmup + steps - 1 and keep_last:
                last = P.Plan(dev, h)
            else:
                P.nlfem_plan_destroy(h)
            desc = {k: v for k, v in kw.items() if k != "mask"}
            log(f"{self.label} {precision} {desc} step {i} {1e3 * (t1 - t0):.1f} ms")
        return times, np.array(tk), info, last, sysm

    def line(self, times, tk, info):
        """pairs/s, ms per step, phase ms and the integration roofline of a run."""
        pairs = int(sum(info["pair_counts"]))
        ms = 1e3 * float(np.mean(times))
        t_int = float(np.mean(tk[:, 3])) * 1e-3
        ach = flops_of(info, self.pb.mc_samples) / t_int / 1e12
        return {"value": round(pairs / (ms * 1e-3), 1), "unit": "pairs/s", "ms_per_step": round(ms, 3),
                "pairs_per_step": pairs, "integrate_ms": round(t_int * 1e3, 3),
                "plan_ms": round(float(np.mean(tk[:, 0])), 3), "rows_ms": round(float(np.mean(tk[:, 4])), 3),
                "integrate_frac_fp64_peak": round(ach / PEAK_FP64_TFLOPS, 4)}


def run_precision(P, mg, dev, args):
    import torch
    pb = mg.precision_problem()
    st = Stepper(P, dev, pb, "precision")

    def run(precision, steps, warmup, strategy="fullcaps", cap_sampling="whole", seed=None, keying="pair"):
        return st.run(precision, steps, warmup, strategy=strategy, cap_sampling=cap_sampling, seed=seed,
                      keying=keying)

    times64, tk64, info, plan64, sys64 = run("fp64", args.steps, args.warmup)
    times32, tk32, info32, plan32, sys32 = run("fp32", args.steps, args.warmup)
    a64 = P.system_to_numpy(sys64)
    a32 = P.system_to_numpy(sys32)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import helpers as H
    e32 = H.value_errors(a32, a64)
    x, it, rr, ok = plan64.solve(sys64, rtol=1e-10)  # first call: work vectors allocated
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    x, it, rr, ok = plan64.solve(sys64, rtol=1e-10)
    torch.cuda.synchronize()
    cg_ms = 1e3 * (time.perf_counter() - c0)
    x32, it32, rr32, ok32 = plan32.solve(sys32, rtol=1e-10)
    xa, xb = x.cpu().numpy(), x32.cpu().numpy()
    sol_err = float(np.max(np.abs(xb - xa)) / max(np.max(np.abs(xa)), 1e-300))
    plan64.destroy()
    plan32.destroy()
    del sys64, sys32, x, x32
    # element keying: N samples per element shared by the outer points
    keyed = {}
    for prec in ([] if args.no_element_keying else ["fp64", "fp32"]):
        ts, tks, inf, pl, sm = run(prec, max(2, args.steps // 2), 1, keying="element")
        pl.destroy()
        del sm
        keyed[prec] = st.line(ts, tks, inf)
    # the plain workload whole, FP64 and FP32-local, solved by CG: compared with
    # the oracle's system and CG solution after the device is closed
    plain = {}
    pbp = mg.plain_problem()
    for prec in ["fp64", "fp32"]:
        pbp.precision = prec
        pl = dev.plan_problem(pbp)
        sm = pl.assemble(pbp.f_qp, pbp.g_nodal)
        xs, its, rrs, oks = pl.solve(sm, rtol=1e-10)
        plain[prec] = (P.system_to_numpy(sm), xs.cpu().numpy())
        pl.destroy()
        del sm

    def plain_vs_oracle(oracle, H):
        pbq = mg.plain_problem()
        So = oracle.problem_assemble(pbq)
        xo, _, _, _ = oracle.cg(So["ff_row_ptr"], So["ff_col"], So["ff_val"], So["rhs"], rtol=1e-12)
        res = {}
        for prec, (g, xg) in plain.items():
            e = H.value_errors(g, So)
            res[prec] = {"max_entry_err_rowscale": max(e["ff_abs"], e["fc_abs"]), "rhs_err": e["rhs"],
                         "solution_err": float(np.max(np.abs(xg - xo)) / max(np.max(np.abs(xo)), 1e-300))}
        return res
    # the library on the outer-tet subset the oracle times (cpu_baseline), kept
    # for the per-entry errors against the oracle
    subset = None
    if not args.no_cpu_baseline:
        mask = mg.outer_subset_mask(pb.mesh.n_tets, args.cpu_fraction, seed=13)
        d_mask = dev.to_dev(mask, torch.uint8)
        subset = {"mask": mask}
        for key, prec, kk in [("fp64", "fp64", "pair"), ("fp32", "fp32", "pair"), ("fp64_element", "fp64", "element")]:
            _, _, _, pl, sm = st.run(prec, 1, 0, keying=kk, mask=d_mask)
            subset[key] = P.system_to_numpy(sm)
            pl.destroy()
            del sm
    # the other ball approximation strategies on the same workload (FP64)
    strategies = None
    if not args.no_strategies:
        strategies = {}
        for sname in ["nocaps", "overlap", "inside", "barycenter"]:
            ts, tks, inf, pl, sm = run("fp64", 2, 1, sname)
            pl.destroy()
            del sm
            npairs = int(sum(inf["pair_counts"]))
            ms = 1e3 * float(np.mean(ts))
            strategies[sname] = {"value": round(npairs / (ms * 1e-3), 1), "unit": "pairs/s", "ms_per_step": round(ms, 3),
                              "pairs_per_step": npairs, "integrate_ms": round(float(np.mean(tks[:, 3])), 3)}
        # fullcaps with the caps sampled on E - U_I (corner tet or three cone tets), and the
        # seed-to-seed spread of the matrix entries in both sampling modes
        ts, tks, inf, pl, sm = run("fp64", 2, 1, "fullcaps", "outside_ui")
        pl.destroy()
        del sm
        npairs = int(sum(inf["pair_counts"]))
        ms = 1e3 * float(np.mean(ts))
        spread = {}
        for mode in ["whole", "outside_ui"]:
            vals = []
            for seed in range(3):
                _, _, _, pl, sm = run("fp64", 1, 0, "fullcaps", mode, seed=seed)
                vals.append(P.system_to_numpy(sm)["ff_val"])
                pl.destroy()
                del sm
            v = np.array(vals)
            spread[mode] = float(np.median(v.std(axis=0) / np.maximum(np.abs(v.mean(axis=0)), 1e-300)))
        strategies["fullcaps_outside_ui"] = {
            "value": round(npairs / (ms * 1e-3), 1), "unit": "pairs/s", "ms_per_step": round(ms, 3),
            "pairs_per_step": npairs, "integrate_ms": round(float(np.mean(tks[:, 3])), 3),
            "entry_seed_spread_median": {k: round(x, 8) for k, x in spread.items()},
            "spread_ratio": round(spread["outside_ui"] / max(spread["whole"], 1e-300), 4)}
    return {"pb": pb, "times64": times64, "tk64": tk64, "times32": times32, "tk32": tk32, "info": info,
            "e32": e32, "sol_err32": sol_err, "cg": {"iters": it, "rel_residual": rr, "converged": bool(ok),
                                                     "ms": round(cg_ms, 2)}, "strategies": strategies,
            "element_keying": keyed, "subset": subset, "plain_vs_oracle": plain_vs_oracle}


def run_large(P, mg, dev, args):
    """The large single-mesh workload: 64^3 Kuhn cubes (1,572,864 tets),
    jitter 0.2h, delta = 4h, N = 128; FP64 and FP32-local, assemble + CG."""
    import torch
    pb = mg.large_problem()
    st = Stepper(P, dev, pb, "large")
    out = {"workload": "64^3 Kuhn cubes (1,572,864 tets), jitter 0.2h seed 1, delta=4h, N=128 MC per cut pair"}
    sysd = {}
    for prec in ["fp64", "fp32"]:
        ts, tks, inf, pl, sm = st.run(prec, args.large_steps, 1)
        line = st.line(ts, tks, inf)
        line["cut_pairs"] = int(sum(inf["pair_counts"][1:]))
        line["in_pairs"] = int(inf["pair_counts"][0])
        line["n_free"] = inf["n_free"]
        line["nnz_ff"] = inf["nnz_ff"]
        x, it, rr, ok = pl.solve(sm, rtol=1e-10)  # first call: work vectors allocated
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        x, it, rr, ok = pl.solve(sm, rtol=1e-10)
        torch.cuda.synchronize()
        line["cg"] = {"iters": it, "rel_residual": rr, "converged": bool(ok),
                      "ms": round(1e3 * (time.perf_counter() - c0), 2)}
        log(f"large {prec}: {line['ms_per_step']:.1f} ms/step, integrate {line['integrate_ms']:.1f} ms, "
            f"CG {it} it {line['cg']['ms']:.1f} ms")
        sysd[prec] = (P.system_to_numpy(sm), x.cpu().numpy())
        out[prec] = line
        pl.destroy()
        del sm, x
        P.nlfem_trim(dev.ctx)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import helpers as H
    e = H.value_errors(sysd["fp32"][0], sysd["fp64"][0])
    xa, xb = sysd["fp64"][1], sysd["fp32"][1]
    out["fp32_local_vs_fp64"] = {"max_entry_err_rowscale": max(e["ff_abs"], e["fc_abs"]), "rhs_err": e["rhs"],
                                 "solution_err": float(np.max(np.abs(xb - xa)) / max(np.max(np.abs(xa)), 1e-300))}
    return out


def run_convergence(P, mg, dev, args):
    """The paper's 3D accuracy experiment (Sec. 5) on synthetic meshes: for
    each strategy and mesh level, the assembly time (plan + numeric, HIP
    synchronised wall clock), a CG solve, the L2(Omega) error against the
    manufactured u, the observed order and the efficiency ratio
    lambda_n = -log(e_{n-1}/e_n) / log(t_{n-1}/t_n)."""
    import torch
    from meshgen import convergence as cv
    levels = [int(v) for v in args.convergence_levels.split(",") if v]
    strategies = ["fullcaps", "nocaps", "barycenter", "overlap", "inside"]
    # fullcaps_exact_g: the same plan with the paper-exact right-hand side (g itself
    # inside the inner integrals over Omega_I) instead of the nodal constraint form
    out = {st: {"m": [], "h": [], "h_avg": [], "l2_error": [], "order": [None], "assembly_ms": [],
                "lambda": [None], "cg_iters": [], "pairs": []} for st in strategies + ["fullcaps_exact_g"]}

    def record(key, m, h_avg, sysm, plan, pb, mesh, t_asm):
        x, it, rr, ok = plan.solve(sysm, rtol=1e-12)
        U = pb.g_nodal.copy()
        U[sysm.free_to_vertex[:sysm.n_free].cpu().numpy()] = x.cpu().numpy()
        err = cv.l2_error(mesh.coords, mesh.tets, pb.tet_region, U)
        r = out[key]
        if r["l2_error"]:
            e0, t_0, h0 = r["l2_error"][-1], r["assembly_ms"][-1] * 1e-3, r["h"][-1]
            r["order"].append(round(math.log(e0 / err) / math.log(h0 / (1.0 / m)), 3))
            r["lambda"].append(round(-math.log(e0 / err) / math.log(t_0 / t_asm), 3))
        r["m"].append(m); r["h"].append(1.0 / m); r["h_avg"].append(round(h_avg, 5))
        r["l2_error"].append(err); r["assembly_ms"].append(round(1e3 * t_asm, 3))
        r["cg_iters"].append(int(it)); r["pairs"].append(int(sum(plan.info["pair_counts"])))
        log(f"convergence m={m} {key}: L2 error {err:.4e}, assembly {1e3 * t_asm:.1f} ms, CG {it} it")
        del x
    for m in levels:
        pb = mg.convergence_problem(m, mc_samples=args.convergence_samples)
        mesh = pb.mesh
        reg = pb.tet_region.astype(bool)
        X = mesh.coords[mesh.tets[reg]]
        edges = [np.linalg.norm(X[:, a] - X[:, b], axis=1) for a in range(4) for b in range(a + 1, 4)]
        h_avg = float(np.mean(edges))
        mm, keep = dev.mesh(mesh.coords, mesh.tets, pb.vertex_free, pb.tet_region)
        d_f = dev.to_dev(pb.f_qp, torch.float64)
        d_g = dev.to_dev(pb.g_nodal, torch.float64)
        for st in strategies:
            prm = P.nlfem_params(pb.delta, pb.psi, pb.mc_samples, pb.seed, P.NLFEM_FP64, None, P.strategy_id(st),
                                 P.cap_sampling_id("whole"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = P.Plan(dev, P.nlfem_plan_create(dev.ctx, mm, prm))
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            sysm = plan.alloc_system()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.nlfem_assemble(plan.handle, d_f, d_g, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val, sysm.fc_row_ptr,
                             sysm.fc_col, sysm.fc_val, sysm.rhs, sysm.free_to_vertex, ctx=dev.ctx)
            torch.cuda.synchronize()
            record(st, m, h_avg, sysm, plan, pb, mesh, t_plan + time.perf_counter() - t1)
            if st == "fullcaps":
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                P.nlfem_assemble_exact_g(plan.handle, d_f, d_g, pb.g_poly, sysm.ff_row_ptr, sysm.ff_col,
                                         sysm.ff_val, sysm.fc_row_ptr, sysm.fc_col, sysm.fc_val, sysm.rhs,
                                         sysm.free_to_vertex, ctx=dev.ctx)
                torch.cuda.synchronize()
                record("fullcaps_exact_g", m, h_avg, sysm, plan, pb, mesh, t_plan + time.perf_counter() - t1)
            plan.destroy()
            del sysm
        del keep, d_f, d_g
    return {"workload": "Omega=(0,1)^3, delta=0.1, u=prod x_d(1-x_d), f=-Lu exact at the outer rule points, "
                        f"g=u nodal; Kuhn meshes h=1/m with a collar of whole cubes, jitter 0.1h; "
                        f"N={args.convergence_samples}; FP64; CG rtol 1e-12",
            "strategies": out,
            "note": "fullcaps_exact_g: fullcaps with the paper-exact right-hand side (g itself in the "
                    "inner integrals over Omega_I); the other lines use nodal g"}


def run_batched(P, mg, dev, args):
    import torch
    pbs = mg.batched_problems(args.batched_count)
    # start from an empty context cache, so the memory figures below are the batch's
    P.nlfem_trim(dev.ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = P.Batch(dev, pbs)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    pairs = int(sum(sum(i["pair_counts"]) for i in b.infos))
    b.set_inputs([p.f_qp for p in pbs], [p.g_nodal for p in pbs])
    t0 = time.perf_counter()
    b.assemble()  # first call: autotune + graph capture + replay
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    ts = []
    for r in range(args.batched_replays):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.assemble()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        log(f"batched replay {r} {1e3 * ts[-1]:.1f} ms")
    tune = b.tuning()
    # with the temporaries the plan builders left in the context's cache, and
    # the batch's own buffers (outputs, plans) once that cache is released
    mem_cached = P.nlfem_memory_in_use(dev.ctx)
    P.nlfem_trim(dev.ctx)
    mem = P.nlfem_memory_in_use(dev.ctx)
    b.destroy()
    P.nlfem_trim(dev.ctx)
    ms = 1e3 * float(np.mean(ts))
    return {"value": round(pairs / (ms * 1e-3), 1), "unit": "pairs/s", "ms_per_replay": round(ms, 2),
            "value_end_to_end": round(pairs / (t_create + ms * 1e-3), 1),
            "end_to_end_note": "pairs / (symbolic phase of all meshes + one graph replay); value: replay only",
            "meshes": len(pbs), "tets": int(sum(p.mesh.n_tets for p in pbs)), "pairs": pairs,
            "dtype": "fp32-local/f64-accumulate", "plan_create_s": round(t_create, 2),
            "first_call_s": round(t_first, 2), "tuned": tune, "device_bytes": int(mem),
            "device_bytes_with_build_cache": int(mem_cached)}


def run_serving(P, mg, args, count, fractions):
    t0 = time.perf_counter()
    reqs = mg.serving_requests(count, rate_per_s=1.0, n_max=40)
    log(f"serving: {count} requests generated in {time.perf_counter() - t0:.1f} s")
    pbs = [r.problem for r in reqs]
    unit_gaps = np.diff([r.arrival_s for r in reqs], prepend=0.0)  # exponential gaps at rate 1/s
    sv = P.Server(0, n_slots=args.slots, pool_bytes=args.pool_gb << 30)
    out = {"requests": count, "slots": args.slots, "pool_gb": args.pool_gb}

    def collect(tickets):
        infos = [sv.wait(tk, 600.0) for tk in tickets]
        for tk in tickets:
            sv.take(tk)
        return infos

    # saturation: everything queued at once
    t0 = time.perf_counter()
    tickets = [sv.submit(pb) for pb in pbs]
    infos = collect(tickets)
    makespan = time.perf_counter() - t0
    pairs = sum(sum(i["pair_counts"]) for i in infos)
    ok = [i for i in infos if i["state"] == 2]
    sat_rate = len(ok) / makespan
    # the largest request (most point pairs) and its service time under the full queue
    big = max(ok, key=lambda i: sum(i["pair_counts"])) if ok else None
    out["saturation"] = {"requests_per_s": round(sat_rate, 3), "pairs_per_s": round(pairs / makespan, 1),
                         "makespan_s": round(makespan, 2), "failed": len(infos) - len(ok),
                         "largest_request_pairs": int(sum(big["pair_counts"])) if big else 0,
                         "largest_request_service_ms": round(1e3 * (big["latency_s"] - big["queue_s"]), 1)
                         if big else None}
    est = np.array([i["est_bytes"] for i in infos], dtype=float)
    peak = np.array([max(i["peak_bytes"], 1) for i in infos], dtype=float)
    out["footprint_est_over_peak"] = {"min": round(float(np.min(est / peak)), 2),
                                      "p50": round(float(np.median(est / peak)), 2),
                                      "max": round(float(np.max(est / peak)), 2)}
    log(f"serving saturation {sat_rate:.2f} req/s, makespan {makespan:.1f} s")
    for frac in fractions:
        rate = frac * sat_rate
        gaps = unit_gaps / rate
        tickets = []
        t0 = time.perf_counter()
        due = t0
        for pb, g in zip(pbs, gaps):
            due += float(g)
            dt = due - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(sv.submit(pb))
        infos = collect(tickets)
        wall = time.perf_counter() - t0
        lat = [1e3 * i["latency_s"] for i in infos if i["state"] == 2]
        # service time: admission to completion (plan, assembly, CG), without the queueing
        svc = [1e3 * (i["latency_s"] - i["queue_s"]) for i in infos if i["state"] == 2]
        pairs = sum(sum(i["pair_counts"]) for i in infos)
        st = sv.stats()
        out[f"poisson_{frac:g}x"] = {
            "rate_per_s": round(rate, 3), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "service_p50_ms": pct(svc, 50), "service_p99_ms": pct(svc, 99),
            "mean_queue_ms": round(1e3 * float(np.mean([i["queue_s"] for i in infos])), 2),
            "requests_per_s": round(len(lat) / wall, 3), "pairs_per_s": round(pairs / wall, 1),
            "max_running": st["max_running"], "failed": len(infos) - len(lat)}
        log(f"serving {frac}x: p50 {pct(lat, 50)} ms p99 {pct(lat, 99)} ms")
    out["pool_peak_gb"] = round(sv.stats()["pool_peak"] / 2**30, 2)
    sv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=0.002)
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--batched-replays", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serving-count", type=int, default=500)
    ap.add_argument("--serving-quick", action="store_true", help="48 requests at 0.9x saturation only")
    ap.add_argument("--no-large", action="store_true", help="skip the 64^3 large workload")
    ap.add_argument("--no-element-keying", action="store_true", help="skip the element-keyed lines")
    ap.add_argument("--large-steps", type=int, default=1)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-strategies", action="store_true", help="skip the nocaps/overlap/inside/barycenter lines")
    ap.add_argument("--no-convergence", action="store_true", help="skip the L2-error convergence study")
    ap.add_argument("--convergence-levels", default="16,20,24,28,32,36,40",
                    help="cubes per unit length m (h = 1/m) of the convergence meshes")
    ap.add_argument("--convergence-samples", type=int, default=64)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--pool-gb", type=int, default=160)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a 256 MiB elementwise copy kernel 3 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding is not part "
              "of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import meshgen as mg
    import paper_2302_07499_amd as P

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        # an elementwise kernel (not a DMA copy, which counters do not see):
        # reads 256 MiB, writes 256 MiB
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("copy calibration: 3 x (256 MiB read + 256 MiB written) by an elementwise kernel")
        del a, b
    log("precision workload")
    dev = P.Device(0)
    pr = run_precision(P, mg, dev, args)
    pb, info = pr["pb"], pr["info"]
    pairs = int(sum(info["pair_counts"]))
    cut = int(sum(info["pair_counts"][1:]))
    inn = int(info["pair_counts"][0])
    ms64 = 1e3 * float(np.mean(pr["times64"]))
    ms32 = 1e3 * float(np.mean(pr["times32"]))
    tk64, tk32 = pr["tk64"], pr["tk32"]

    # roofline of the dominant kernel (pair integration), from HIP events on the library's stream
    t_int = float(np.mean(tk64[:, 3])) * 1e-3
    flops = FLOP_PER_SAMPLE * cut * pb.mc_samples + FLOP_PER_CUT_PAIR * cut + FLOP_PER_IN_PAIR * inn
    achieved = flops / t_int / 1e12
    traffic, tinfo = recorded_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_integrate<double, false, 0>", "kernel_ms": round(t_int * 1e3, 3)}
    if traffic is None:
        roofline["traffic_note"] = tinfo
    else:
        roofline.update(tinfo)
    valu = recorded_valu()
    if valu is not None:
        # hardware view from the counters: VALU wave instructions per SIMD-cycle
        # against the issue limit, and the FP64 FLOPs the hardware executed
        roofline["valu_issue_frac"] = round(valu["issue_frac"], 4)
        roofline["hw_f64_tflops"] = round(valu["hw_f64_flop_per_launch"] / t_int / 1e12, 3)

    convergence = None
    if not args.no_convergence:
        log("convergence workload")
        convergence = run_convergence(P, mg, dev, args)
        P.nlfem_trim(dev.ctx)

    batched = None
    if not args.no_batched:
        log("batched workload")
        batched = run_batched(P, mg, dev, args)
    P.nlfem_trim(dev.ctx)

    large = None
    if not args.no_large:
        log("large workload")
        large = run_large(P, mg, dev, args)
        P.nlfem_trim(dev.ctx)
    dev.close()

    serving = None
    if not args.no_serving:
        count = 48 if args.serving_quick else args.serving_count
        fractions = [0.9] if args.serving_quick else [0.5, 0.9]
        serving = run_serving(P, mg, args, count, fractions)

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        sub = pr["subset"]
        mask = sub["mask"]
        region = np.array([pb.vertex_free[tt].any() for tt in pb.mesh.tets])
        n_outer = int((mask.astype(bool) & region).sum())
        log(f"oracle on {n_outer} outer tets")
        c0 = time.perf_counter()
        S = oracle.problem_assemble(pb, outer_mask=mask)
        dt = time.perf_counter() - c0
        opairs = int(S["pair_counts"].sum())
        cpu = {"value": round(opairs / dt, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"precision workload, {n_outer} of {int(region.sum())} outer tets "
                         f"(seeded subset), {opairs} pairs in {dt:.1f} s, serial FP64 brute force",
               "host": host_cpu()}
        # the library's results on the same subset against the oracle's: per-entry
        # error (after the near-tie allowance) and the CG solution error
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import helpers as H
        vs_oracle = {"subset": f"precision workload, {n_outer} outer tets", "near_ties": int(S["near_ties"])}
        for key in ["fp64", "fp32"]:
            e = H.value_errors(sub[key], S)
            vs_oracle[key] = {"max_entry_err_rowscale": max(e["ff_abs"], e["fc_abs"]),
                              "max_entry_rel_err": max(e["ff_rel"], e["fc_rel"]), "rhs_err": e["rhs"]}
        # whole systems and CG solutions: the plain workload, against the oracle
        vs_oracle["plain_solution"] = pr["plain_vs_oracle"](oracle, H)
        # element keying against the element-keyed oracle
        pbe = mg.precision_problem()
        pbe.keying = "element"
        Sk = oracle.problem_assemble(pbe, outer_mask=mask)
        e = H.value_errors(sub["fp64_element"], Sk)
        vs_oracle["fp64_element"] = {"max_entry_err_rowscale": max(e["ff_abs"], e["fc_abs"]),
                                     "max_entry_rel_err": max(e["ff_rel"], e["fc_rel"]), "rhs_err": e["rhs"]}

    lat = np.array(pr["times64"]) * 1e3
    e32 = pr["e32"]
    out = {
        "metric": "assembled element-pairs/s (FP32-local vs FP64) at stated err; p50/p99 latency",
        "value": round(pairs / (ms64 * 1e-3), 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "precision: 32^3 Kuhn cubes (196,608 tets), jitter 0.2h seed 1, delta=3h, "
                               "N=64 MC per cut pair, assemble (plan+numeric), CG timed apart",
                   "pairs_per_step": pairs, "cut_pairs": cut, "in_pairs": inn,
                   "mc_samples_per_step": cut * pb.mc_samples, "n_free": info["n_free"],
                   "nnz_ff": info["nnz_ff"], "nnz_fc": info["nnz_fc"]},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "fp32_local": {"value": round(pairs / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 3),
                       "max_entry_err_vs_fp64_rowscale": max(e32["ff_abs"], e32["fc_abs"]),
                       "rhs_err_vs_fp64": e32["rhs"], "solution_err_vs_fp64": pr["sol_err32"],
                       "kernel_ms": round(float(np.mean(tk32[:, 3])), 3)},
        "phases_ms_fp64": {"plan": round(float(np.mean(tk64[:, 0])), 3),
                           "classify": round(float(np.mean(tk64[:, 1])), 3),
                           "pattern": round(float(np.mean(tk64[:, 2])), 3),
                           "integrate": round(float(np.mean(tk64[:, 3])), 3),
                           "rows": round(float(np.mean(tk64[:, 4])), 3),
                           "assemble": round(float(np.mean(tk64[:, 5])), 3)},
        "element_keying": pr["element_keying"],
        "errors_vs_oracle_subset": vs_oracle,
        "cg": pr["cg"],
        "strategies_fp64": pr["strategies"],
        "convergence": convergence,
        "batched": batched,
        "large": large,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
