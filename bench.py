#!/usr/bin/env python3
"""Benchmark of one EnKF analysis step on one MI355X.

A step is the whole hot path on one batch of synthetic input already resident
in HBM: V and D from the background ensemble, the factorisation of
(R + V V^T) by the iterative Sherman-Morrison formula, the solve for Z and the
analysis update X^A. Default workload: the Lorenz-96 ring with n_state =
1,048,576, N = 96 members, every 4th variable observed (n_obs = 262,144),
R = diag(U(0.005, 0.02)), plain FP64.

Prints ONE JSON line (rank 0) with the throughput in analysis solves/s, the
roofline record of the dominant kernel (the per-level solve sweep, HBM-bound)
and the FP64 CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "analysis solves/sec + HBM GB/s or MFMA TFLOP/s, mixed vs plain FP64 at stated residual"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--n-state", type=int, default=1_048_576)
    ap.add_argument("--n-ens", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the analysis path is built and timed on a single MI355X; "
              "sharding across GPUs is described in DESIGN.md but not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1302_3876_amd as pk
    import synth

    t0 = time.time()
    w = synth.c2(n_state=args.n_state, n_ens=args.n_ens)
    print(f"[bench] inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    es = 8 if args.dtype == "f64" else 4
    XB = pk.to_colmajor(w.XB, dtype=tdt)
    E = pk.to_colmajor(w.E, dtype=tdt)
    obs = torch.as_tensor(w.obs_idx).cuda()
    y = torch.as_tensor(w.y).cuda()
    r = torch.as_tensor(w.r).cuda()
    n_state, N, n_obs = w.n_state, w.n_ens, w.n_obs
    V = pk.colmajor(n_obs, N, tdt)
    D = pk.colmajor(n_obs, N, tdt)
    Z = pk.colmajor(n_obs, N, tdt)
    XA = pk.colmajor(n_state, N, tdt)

    pk.enkf_build_vd(XB, obs, y, E, V, D)
    plan = pk.Plan(r, V)

    def step():
        pk.enkf_build_vd(XB, obs, y, E, V, D)
        plan.refactor(r, V)
        plan.solve(D, Z)
        plan.analysis(XB, Z, XA)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    info = plan.info()   # raises if a kernel latched an error

    # timed region: K whole steps, bracketed by device synchronisation
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    print(f"[bench] {args.steps} steps in {ms_total:.2f} ms (host wall {wall * 1e3:.2f} ms)", file=sys.stderr,
          flush=True)

    # per-kernel durations with HIP events on the plan's stream (the current
    # stream), over K more steps of the same workload
    plan.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kc = {c: plan.timing(c) for c in ("factor_sweep", "solve_sweep", "analysis", "gram")}
    plan.set_timing(False)
    sw = kc["solve_sweep"]
    avg_ms = sw["ms"] / max(sw["launches"], 1)
    bytes_per_launch = sw["bytes"] / max(sw["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "level_kernel (solve sweep, one launch per level)",
                "avg_launch_us": round(avg_ms * 1e3, 2), "alg_bytes_per_launch": bytes_per_launch}
    breakdown = {}
    for c, d in kc.items():
        per = d["ms"] / args.steps
        breakdown[c] = {"ms_per_step": round(per, 4), "launches_per_step": d["launches"] // args.steps,
                        "GB/s": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9, 1) if d["ms"] > 0 else None,
                        "TFLOP/s": round(d["flops"] / (d["ms"] * 1e-3) / 1e12, 3) if d["ms"] > 0 else None}

    # accuracy of this step's solve, from the device result (host FP64 check)
    cpu_baseline = None
    relres = None
    if not args.no_cpu_baseline:
        import oracle
        Zh = Z.cpu().numpy().astype(np.float64)
        Vh = V.cpu().numpy().astype(np.float64)
        Dh = D.cpu().numpy().astype(np.float64)
        relres = oracle.rel_residual(w.r, Vh, Zh, Dh)
        # the oracle on the host: whole steps of the same workload until the
        # budget is used (at least one)
        XBh = XB.cpu().numpy().astype(np.float64)
        Eh = E.cpu().numpy().astype(np.float64)
        reps, c0 = 0, time.perf_counter()
        while True:
            Vo, Do = oracle.build_vd(XBh, w.obs_idx, w.y, Eh)
            Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
            oracle.analysis(XBh, Vo, Zo)
            reps += 1
            el = time.perf_counter() - c0
            if el >= args.cpu_budget_s or reps >= 5:
                break
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        cpu_baseline = {"value": round(reps / el, 4), "unit": "solves/s", "cores": threads, "kind": "oracle",
                        "sample": f"{reps} whole analysis step(s) (build V,D + solve + analysis) of the same "
                                  f"workload in FP64, {el:.1f} s"}

    value = 1000.0 / ms_per_step
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded Lorenz-96 ensemble, perturbed observations)",
        "config": {"workload": f"Lorenz-96 ring n_state={n_state}, N={N}, n_obs={n_obs} (every 4th variable), "
                               f"R=diag(U(0.005,0.02)); plain iterative Sherman-Morrison; step = build V,D + "
                               f"factor + solve + analysis update",
                   "n_state": n_state, "n_ens": N, "n_obs": n_obs, "algo": "plain", "storage": args.dtype},
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        "kernels": breakdown,
        "rel_residual": relres,
        "gamma_range": [info["gamma_min"], info["gamma_max"]],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
