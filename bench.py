#!/usr/bin/env python3
"""Benchmark: assembled (point, element) pairs per second of the fullcaps
assembly on one MI355X, FP64 and FP32-local.

Workload: 32^3 Kuhn-split cubes of [0,1]^3 (196,608 tets, 35,937 vertices),
interior vertices jittered uniformly by +-0.2h (seed 1), delta = 3h,
psi = 15/(4 pi delta^5), N = 64 Monte Carlo samples per cut pair, f = -2,
g = x1^2.  One step is one pass of the whole assembly path on the device:
mesh layout, cell list, exact classification, local vertex sets and the
sorted-key reduction plan (plan_create), then pair integration, reductions
and the right-hand side (assemble).  Inputs are resident in HBM when the
timed region starts; the CG solve is timed separately.

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


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fraction", type=float, default=0.0008)
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
    log("building inputs")
    pb = mg.precision_problem()
    mesh = pb.mesh
    dev = P.Device(0)
    t = torch
    d_coords = dev.to_dev(mesh.coords, t.float64)
    d_tets = dev.to_dev(mesh.tets, t.int32)
    d_free = dev.to_dev(pb.vertex_free, t.uint8)
    d_f = dev.to_dev(pb.f_qp, t.float64)
    d_g = dev.to_dev(pb.g_nodal, t.float64)
    m = P.nlfem_mesh(mesh.n_vertices, mesh.n_tets, d_coords.data_ptr(), d_tets.data_ptr(), d_free.data_ptr(),
                     None, 1)

    def run(precision, steps, warmup):
        prm = P.nlfem_params(pb.delta, pb.psi, pb.mc_samples, pb.seed,
                             P.NLFEM_FP32_LOCAL if precision == "fp32" else P.NLFEM_FP64, None)
        # allocate outputs once (sizes are the same every step)
        plan = P.Plan(dev, P.nlfem_plan_create(dev.ctx, m, prm))
        sysm = plan.alloc_system()
        plan.destroy()
        times, tk = [], []
        info = None
        for i in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = P.nlfem_plan_create(dev.ctx, m, prm)
            P.nlfem_assemble(h, d_f, d_g, sysm.ff_row_ptr, sysm.ff_col, sysm.ff_val, sysm.fc_row_ptr, sysm.fc_col,
                             sysm.fc_val, sysm.rhs, sysm.free_to_vertex, ctx=dev.ctx)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if i >= warmup:
                times.append(t1 - t0)
                tk.append(P.nlfem_plan_timings(h))
            if info is None:
                info = P.nlfem_plan_info(h)
            if i == warmup + steps - 1:
                plan = P.Plan(dev, h)
            else:
                P.nlfem_plan_destroy(h)
            log(f"{precision} step {i} {1e3 * (t1 - t0):.1f} ms")
        return times, np.array(tk), info, plan, sysm

    times64, tk64, info, plan64, sys64 = run("fp64", args.steps, args.warmup)
    times32, tk32, info32, plan32, sys32 = run("fp32", args.steps, args.warmup)
    pairs = int(sum(info["pair_counts"]))
    cut = int(sum(info["pair_counts"][1:]))
    inn = int(info["pair_counts"][0])
    ms64 = 1e3 * float(np.mean(times64))
    ms32 = 1e3 * float(np.mean(times32))

    # FP32-local vs FP64 per-entry difference (relative to the row scale)
    a64 = P.system_to_numpy(sys64)
    a32 = P.system_to_numpy(sys32)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import helpers as H
    e32 = H.value_errors(a32, a64)

    # CG (timed separately)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    x, it, rr, ok = plan64.solve(sys64, rtol=1e-10)
    torch.cuda.synchronize()
    cg_ms = 1e3 * (time.perf_counter() - c0)

    # roofline of the dominant kernel (pair integration), from HIP events on the library's stream
    t_int = float(np.mean(tk64[:, 3])) * 1e-3
    flops = FLOP_PER_SAMPLE * cut * pb.mc_samples + FLOP_PER_CUT_PAIR * cut + FLOP_PER_IN_PAIR * inn
    achieved = flops / t_int / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "kernel": "k_integrate<double>", "kernel_ms": round(t_int * 1e3, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        mask = mg.outer_subset_mask(mesh.n_tets, args.cpu_fraction, seed=13)
        region = np.array([pb.vertex_free[tt].any() for tt in mesh.tets])
        n_outer = int((mask.astype(bool) & region).sum())
        log(f"oracle on {n_outer} outer tets")
        c0 = time.perf_counter()
        S = oracle.problem_assemble(pb, outer_mask=mask)
        dt = time.perf_counter() - c0
        opairs = int(S["pair_counts"].sum())
        cpu = {"value": round(opairs / dt, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"precision workload, {n_outer} of {int(region.sum())} outer tets "
                         f"(seeded subset), {opairs} pairs in {dt:.1f} s, serial FP64 brute force"}

    lat = np.array(times64) * 1e3
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
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "fp32_local": {"value": round(pairs / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 3),
                       "max_entry_err_vs_fp64_rowscale": max(e32["ff_abs"], e32["fc_abs"]),
                       "rhs_err_vs_fp64": e32["rhs"],
                       "kernel_ms": round(float(np.mean(tk32[:, 3])), 3)},
        "phases_ms_fp64": {"plan": round(float(np.mean(tk64[:, 0])), 3), "classify": round(float(np.mean(tk64[:, 1])), 3),
                           "pattern_sort": round(float(np.mean(tk64[:, 2])), 3),
                           "integrate": round(float(np.mean(tk64[:, 3])), 3),
                           "reduce": round(float(np.mean(tk64[:, 4])), 3),
                           "assemble": round(float(np.mean(tk64[:, 5])), 3)},
        "cg": {"iters": it, "rel_residual": rr, "converged": bool(ok), "ms": round(cg_ms, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    plan64.destroy()
    plan32.destroy()
    dev.close()


if __name__ == "__main__":
    main()
