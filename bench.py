#!/usr/bin/env python3
"""Benchmark of the EnKF analysis on one MI355X.

Default workload (the headline line), the mixed-precision configuration:
n_obs = 2,097,152 observations, N = 256 members, V_ij = g_ij s_i/sqrt(255)
(g ~ N(0,1), s_i ~ U(0.5, 2)), R = diag(U(0.01, 0.1)), D ~ N(0, 1). A step
is one analysis solve on inputs already resident in HBM: the factorisation
of (R + V V^T) and the solve for Z (with every refinement step). The forms:
blocked solves with FP32, BF16x3 and FP16x2 panels refined in FP64 to a
relative residual of 1e-10 (the mixed forms; FP32 panels also at the
configuration's b = 64), blocked FP64 with and without one FP64 refinement
step, and the plain level-by-level FP64 iteration. Panel widths not given
are picked by the library's tuner (ENKF_FLAG_AUTOTUNE). Each form's
residual and backward error are formed on the host from the returned Z.
`value` is the solves/s of the fastest mixed form that meets its gate; the
line also carries every form, the speedups over plain FP64 of the forms that
meet their gates, and the roofline of the headline form's dominant kernel.

--workload c2: the Lorenz-96 ring with n_state = 1,048,576, N = 96, every
4th variable observed; a step is build + factor + solve + analysis.
--workload c1: the 40-variable Lorenz-96 step, latency per analysis (eager
launches and one HIP graph replay). c4, c5, loc and cycle: see --help.

Prints ONE JSON line with the roofline record and the FP64 CPU oracle timed
on the host as a baseline.
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
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # vector FMA rates (published)
METRIC = "analysis solves/sec + HBM GB/s or MFMA TFLOP/s, mixed vs plain FP64 at stated residual"
CLASSES = ("factor_sweep", "solve_sweep", "build", "analysis", "gram", "panel_update", "panel_factor", "residual",
           "step1", "fused_sweep", "residual_tn")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5", "loc", "cycle"], default="c3",
                    help="c3 (default): mixed vs plain FP64 solves at n_obs=2^21, N=256; c1: 40-variable latency; "
                         "c2: Lorenz-96 n_state=2^20, N=96 full step; c4: 4096 localized analyses; c5: N=1024 "
                         "FP32 ensemble; loc: partial localization; cycle: Lorenz-96 cycling filter")
    ap.add_argument("--forms", default="", help="comma list; default: every form of the workload; "
                                                 "FORM@b fixes the panel width of a blocked form")
    ap.add_argument("--block", type=int, default=0, help="panel width of the blocked forms without @b "
                                                         "(0: the library's tuner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cycle-shapes", action="store_true", help="cycle workload: skip the shape sweep")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    ap.add_argument("--calibrate-mfma", action="store_true",
                    help="print the measured matrix-core throughput (enkf_mfma_peak) per input type and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 4 times (the known-size kernel that scales the HBM "
                         "byte counters) and exit")
    return ap.parse_args()


FORMS = {
    # name: (algo, storage, math, refine)
    "plain_f64": ("plain", "f64", "f64", 0),
    "plain_f32": ("plain", "f32", "f32", 0),
    "plain_f64_pivot": ("plain", "f64", "f64", 0),
    "plain_f64_blockr4": ("plain", "f64", "f64", 0),
    "blocked_f64": ("blocked", "f64", "f64", 0),
    "blocked_f32": ("blocked", "f32", "f32", 0),
    "blocked_f64_refined": ("blocked", "f64", "f64", 1),
    "mixed_f32": ("blocked", "f64", "f32", 8),
    "mixed_bf16x3": ("blocked", "f64", "bf16x3", 12),
    "mixed_f16x2": ("blocked", "f64", "f16x2", 12),
}
DEFAULT_FORMS = {"c2": ["plain_f64", "plain_f32", "blocked_f64", "blocked_f64_refined", "mixed_f32", "plain_f64_pivot",
                        "plain_f64_blockr4"],
                 "c3": ["mixed_f32", "mixed_f32@64", "mixed_bf16x3", "mixed_f16x2", "blocked_f64",
                        "blocked_f64_refined", "plain_f64"]}
MIXED_GATE = 1e-10      # relative residual the mixed forms refine to
FP64_ETA_GATE = 1e-12   # normwise backward error of the FP64 forms


def form_spec(name):
    """'mixed_f32@64' -> ('mixed_f32', 64); no '@': (name, 0)."""
    base, _, b = name.partition("@")
    return base, int(b) if b else 0


def gpu_inputs(w, dtype, pk, torch):
    d = {"r": torch.as_tensor(w.r).cuda()}
    if w.XB is not None:
        d["XB"] = pk.to_colmajor(w.XB, dtype=dtype)
        d["E"] = pk.to_colmajor(w.E, dtype=dtype)
        d["obs"] = torch.as_tensor(w.obs_idx).cuda()
        d["y"] = torch.as_tensor(w.y).cuda()
        d["V"] = pk.colmajor(w.n_obs, w.n_ens, dtype)
        d["D"] = pk.colmajor(w.n_obs, w.n_ens, dtype)
        d["XA"] = pk.colmajor(w.n_state, w.n_ens, dtype)
    else:
        d["V"] = pk.to_colmajor(w.V, dtype=dtype)
        d["D"] = pk.to_colmajor(w.D, dtype=dtype)
    d["Z"] = pk.colmajor(w.n_obs, w.n_ens, dtype)
    return d


def cpu_model() -> str:
    """The host processor's model name (the cores the oracle ran on)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_steps(torch, step, steps):
    """Time `steps` calls of step() with HIP events on the current stream (the
    one the library launches on): one event before the first step and one
    after each. Returns (mean, median, min) milliseconds per step; the mean is
    over the whole bracket."""
    import numpy as np
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[-1]) / steps, float(np.median(per)), float(min(per))


def run_form(name, w, args, pk, torch, cache, wnorm=None):
    import numpy as np
    base_name, fixed_b = form_spec(name)
    algo, storage, math, refine = FORMS[base_name]
    tdt = torch.float64 if storage == "f64" else torch.float32
    if storage not in cache:
        cache.clear()
        torch.cuda.empty_cache()
        cache[storage] = gpu_inputs(w, tdt, pk, torch)
    g = cache[storage]
    full = "XB" in g
    if full:
        pk.enkf_build_vd(g["XB"], g["obs"], g["y"], g["E"], g["V"], g["D"])
    block = (fixed_b or args.block) if algo == "blocked" else 0
    # mixed forms stop once the FP64 residual is <= 1e-10, checked
    # synchronously per refinement step, at most `refine` steps; FP64 panels
    # take exactly `refine` correction steps
    tol = (0.0 if math == "f64" else MIXED_GATE) if refine else 0.0
    block_r = None
    if name.endswith("_blockr4"):
        # R block diagonal, blocks of 4 neighbouring observations with
        # correlation 0.5^|i-j| and the diagonal r: R_b = D^(1/2) C D^(1/2)
        rh = g["r"].cpu().numpy()
        nb = w.n_obs // 4
        idx = np.arange(4)
        C = 0.5 ** np.abs(idx[:, None] - idx[None, :])
        sd = np.sqrt(rh[: nb * 4].reshape(nb, 4))
        Rb = sd[:, :, None] * C[None] * sd[:, None, :]
        packed = np.ascontiguousarray(Rb.transpose(0, 2, 1)).ravel()      # column-major per block
        block_r = (np.arange(0, w.n_obs + 1, 4, dtype=np.int64), torch.as_tensor(packed).cuda())
    plan = pk.Plan(g["r"], g["V"], algo=algo, math=math, block=block, refine_max_iter=refine, refine_tol=tol,
                   pivot=base_name.endswith("_pivot"), block_r=block_r, autotune=(algo == "blocked" and block == 0))
    tuning = plan.tuning()
    last = {}

    def step():
        if full:
            pk.enkf_build_vd(g["XB"], g["obs"], g["y"], g["E"], g["V"], g["D"])
        # factorisation + solve in one call (plain: one level loop over U and Z)
        if block_r is not None:
            plan.refactor_block_r(block_r[1], g["V"])
            plan.solve(g["D"], g["Z"])
        elif refine:
            _, last["info"] = plan.factor_solve(g["r"], g["V"], g["D"], g["Z"], info=True)
        else:
            plan.factor_solve(g["r"], g["V"], g["D"], g["Z"])
        if full:
            plan.analysis(g["XB"], g["Z"], g["XA"])

    steps = args.steps if not (base_name == "plain_f64" and args.workload == "c3") else max(2, args.steps // 10)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    info = plan.info()
    ms, ms_med, ms_min = timed_steps(torch, step, steps)
    print(f"[bench] {name}: {ms:.3f} ms/step over {steps} steps", file=sys.stderr, flush=True)
    # per-kernel durations, HIP events on the plan's stream, same workload
    plan.set_timing(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kern = {}
    for c in CLASSES:
        t = plan.timing(c)
        if t["launches"] == 0:
            continue
        kern[c] = {"ms_per_step": round(t["ms"] / steps, 4), "launches_per_step": t["launches"] // steps,
                   "avg_launch_us": round(1e3 * t["ms"] / t["launches"], 2),
                   "alg_bytes_per_launch": t["bytes"] / t["launches"],
                   "alg_flops_per_launch": t["flops"] / t["launches"],
                   "GB/s": round(t["bytes"] / (t["ms"] * 1e-3) / 1e9, 1) if t["ms"] > 0 else None,
                   "TFLOP/s": round(t["flops"] / (t["ms"] * 1e-3) / 1e12, 3) if t["ms"] > 0 else None}
    plan.set_timing(False)
    # accuracy of the device result: FP64 residual of the system solved,
    # formed on the host with numpy (a diagnostic, not part of the path)
    Vh = np.asfortranarray(g["V"].cpu().numpy().astype(np.float64))
    Dh = np.asfortranarray(g["D"].cpu().numpy().astype(np.float64))
    Zh = np.asfortranarray(g["Z"].cpu().numpy().astype(np.float64))
    if block_r is not None:
        RZ = np.einsum("bij,bjm->bim", Rb, Zh.reshape(-1, 4, Zh.shape[1])).reshape(Zh.shape)
        rho = Dh - RZ - Vh @ (Vh.T @ Zh)
    else:
        rho = Dh - w.r[:, None] * Zh - Vh @ (Vh.T @ Zh)
    dn, zn = float(np.linalg.norm(Dh)), float(np.linalg.norm(Zh))
    relres = float(np.linalg.norm(rho)) / dn
    # normwise backward error with the oracle's ||W||_2 estimate (FP64 forms)
    eta = float(np.linalg.norm(rho)) / (wnorm * zn + dn) if wnorm else None
    del Vh, Dh, Zh, rho
    if math == "f64":
        gate = {"kind": f"FP64: eta <= {FP64_ETA_GATE:g}", "met": eta is not None and eta <= FP64_ETA_GATE}
    elif storage == "f64":
        gate = {"kind": f"mixed: relres <= {MIXED_GATE:g}", "met": relres <= MIXED_GATE}
    else:
        gate = {"kind": "FP32 storage: none stated", "met": None}
    out = {"ms_per_step": round(ms, 4), "ms_median": round(ms_med, 4), "ms_min": round(ms_min, 4),
           "solves_per_s": round(1000.0 / ms, 3), "algo": algo, "storage": storage,
           "math": math, "refine_iters": last["info"]["refine_iters"] if refine else 0,
           "device_rel_residual": last["info"]["rel_residual"] if refine else None,
           "block": info["block"], "block_tuning_ms": tuning or None,
           "rel_residual": relres, "backward_error": eta, "gate": gate,
           "gamma_range": [info["gamma_min"], info["gamma_max"]], "kernels": kern}
    plan.close()
    return out


def traffic_record(source_rel: str, kernel: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary under
    profiles/ (FETCH_SIZE + WRITE_SIZE, calibrated with a copy of known size),
    or None once the kernel source no longer has the hash they were taken at."""
    import glob
    import hashlib
    src = os.path.join(ROOT, source_rel)
    if not os.path.exists(src):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if line.startswith("traffic-record:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("source") == source_rel and rec.get("source_sha256") == sha and rec.get("kernel") == kernel:
                    return rec["bytes_per_launch"]
    return None


def roofline_of(form, name):
    k = form["kernels"]
    if form["algo"] == "plain":
        # the dominant class: the Z-sweep (when the U and Z loops run
        # separately, which the library picks when their joint working set
        # would overflow the last-level cache) or the fused sweep
        fused = "fused_sweep" in k
        c = k["fused_sweep" if fused else "solve_sweep"]
        ach = c["alg_bytes_per_launch"] / (c["avg_launch_us"] * 1e-6) / 1e9
        # (the last two template arguments: a block walks several row tiles,
        # streamed columns; c3 takes the streamed instance, one tile per block)
        names = (["level_kernel<double, 2, false, true, true, false, true>",
                  "level_kernel<double, 2, false, true, true, false, false>"] if fused else
                 ["level_kernel<double, 2, false, true, false, false, false>"])
        traffic = None
        for kn in names if name == "plain_f64" else []:
            traffic = traffic or traffic_record("paper_1302_3876_amd/csrc/level_kernels.hip", kn)
        what = "fused factor + solve sweep" if fused else "solve sweep (Z columns)"
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"level_kernel ({name}: {what}, one launch per level)",
                "avg_launch_us": c["avg_launch_us"], "alg_bytes_per_launch": c["alg_bytes_per_launch"]}
    # blocked and mixed forms: the kernel class with the most time per step
    # (the panel products, the panel updates, or the two FP64 products of
    # the refinement residual), rated against the matrix-core peak of the
    # type it runs in
    mf = {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16", "bf16x3": "bf16", "f16x2": "f16"}[form["math"]]
    lowp = form["math"] in ("bf16", "f16", "bf16x3", "f16x2")
    wt = "double" if form["storage"] == "f64" and form["math"] == "f64" else "float"
    names = {
        "gram": ("f64" if form["math"] == "f64" else mf,
                 f"tn_lowp_kernel<{form['math']}> (panel products V_K^T X)" if lowp else
                 f"tn_partial_kernel<{wt}> (panel products V_K^T X)"),
        "panel_update": ("f64" if form["math"] == "f64" else mf,
                         f"nn_lowp_kernel<{form['math']}, UPDATE> (panel update X -= U_K Q)" if lowp else
                         f"nn_kernel<{wt}, UPDATE> (panel update X -= U_K Q)"),
        "residual": ("f64", "nn_kernel<double, RESIDUAL> (FP64 residual D - (R Z + V G))"),
        "residual_tn": ("f64", "tn_partial_kernel<double> (FP64 residual product G = V^T Z)"),
    }
    cls = max((c for c in names if c in k), key=lambda c: k[c]["ms_per_step"])
    c = k[cls]
    peak_t, kname = names[cls]
    ach = c["alg_flops_per_launch"] / (c["avg_launch_us"] * 1e-6) / 1e12
    peak = MFMA_PEAK_TFLOPS[peak_t]
    return {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
            "traffic": traffic_record("paper_1302_3876_amd/csrc/gemm_mfma.hip", kname.split(" (")[0])
            if cls in ("residual", "residual_tn") else None,
            "kernel": f"{kname}, {name}", "kernel_class": cls, "peak_type": peak_t,
            "share_of_step": round(c["ms_per_step"] / form["ms_per_step"], 3),
            "avg_launch_us": c["avg_launch_us"], "alg_flops_per_launch": c["alg_flops_per_launch"],
            "alg_bytes_per_launch": c["alg_bytes_per_launch"]}


def cpu_baseline(w, args):
    """The FP64 oracle on the host. c2: whole analysis steps of the same
    workload. c3: the solve on the first n/32 observations (the solve costs
    3(N^2 n + N n) operations, linear in n), scaled to the full n."""
    import oracle
    reps, c0 = 0, time.perf_counter()
    scale = 1.0
    if w.XB is None:
        ns = max(1, w.n_obs // 32)
        scale = w.n_obs / ns
        r_s, V_s, D_s = w.r[:ns].copy(), w.V[:ns].copy(order="F"), w.D[:ns].copy(order="F")
        c0 = time.perf_counter()
    while True:
        if w.XB is not None:
            Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
            Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
            oracle.analysis(w.XB, Vo, Zo)
        else:
            oracle.sm_solve(r_s, V_s, D_s)
        reps += 1
        el = time.perf_counter() - c0
        if el >= args.cpu_budget_s or reps >= 5:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    if w.XB is not None:
        what = f"{reps} whole analysis step(s) (build V,D + solve + analysis) of the same workload, FP64, {el:.1f} s"
    else:
        what = (f"{reps} solve(s) on the first {w.n_obs // 32} of {w.n_obs} observations, FP64, {el:.1f} s, "
                f"time scaled by {scale:.0f} (cost linear in n)")
    return {"value": round(reps / (el * scale), 5), "unit": "solves/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": what}


def run_c1(args, pk, torch):
    """c1: one FP64 analysis step of the 40-variable Lorenz-96 ensemble (N =
    20, every other variable observed): build V and D, factor and solve by the
    plain level iteration, analysis update. Latency per step with eager
    launches and with the same step captured once in a HIP graph and
    replayed. The plan and the capture live on a side stream (the plan's
    stream is fixed at init)."""
    import numpy as np
    import oracle
    import synth
    w = synth.c1()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        XB = pk.to_colmajor(w.XB)
        E = pk.to_colmajor(w.E)
        obs = torch.as_tensor(w.obs_idx).cuda()
        y = torch.as_tensor(w.y).cuda()
        r = torch.as_tensor(w.r).cuda()
        V, D = pk.enkf_build_vd(XB, obs, y, E)
        Z = pk.colmajor(w.n_obs, w.n_ens)
        XA = pk.colmajor(w.n_state, w.n_ens)
        plan = pk.Plan(r, V)

        def step():
            pk.enkf_build_vd(XB, obs, y, E, V, D)
            plan.factor_solve(r, V, D, Z)
            plan.analysis(XB, Z, XA)
        for _ in range(max(args.warmup, 3)):
            step()
        steps = max(args.steps, 200)
        ms_e, med_e, min_e = timed_steps(torch, step, steps)
        xa_eager = XA.cpu().numpy()
        g = torch.cuda.CUDAGraph()
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            step()
        XA.zero_()
        for _ in range(3):
            g.replay()
        ms_g, med_g, min_g = timed_steps(torch, g.replay, steps)
        xa_graph = XA.cpu().numpy()
    s.synchronize()
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    XAo = oracle.analysis(w.XB, Vo, oracle.sm_solve(w.r, Vo, Do)["Z"])
    inc_err = float(np.max(np.abs((xa_graph - w.XB) - (XAo - w.XB))) / np.max(np.abs(XAo - w.XB)))
    res = {"eager": {"ms_per_step": round(ms_e, 5), "ms_median": round(med_e, 5), "ms_min": round(min_e, 5),
                     "analyses_per_s": round(1e3 / ms_e, 1)},
           "graph": {"ms_per_step": round(ms_g, 5), "ms_median": round(med_g, 5), "ms_min": round(min_g, 5),
                     "analyses_per_s": round(1e3 / ms_g, 1)},
           "graph_equals_eager_bitwise": bool(np.array_equal(xa_graph, xa_eager)),
           "max_increment_err_vs_oracle": inc_err}
    plan.close()
    return w, res


def run_local(w, args, pk, torch):
    """c4: every local analysis in one launch (a HIP graph replay)."""
    import numpy as np
    import oracle
    start, ln, pts = w.extra["win_start"], w.extra["win_len"], w.extra["state_idx"]
    # V and D of the whole ring built on the device from the FP32 ensemble
    XBd = pk.to_colmajor(w.XB.astype(np.float32), dtype=torch.float32)
    Ed = pk.to_colmajor(w.E.astype(np.float32), dtype=torch.float32)
    Vd, Dd = pk.enkf_build_vd(XBd, torch.as_tensor(w.obs_idx).cuda(), torch.as_tensor(w.y).cuda(), Ed)
    r = torch.as_tensor(w.r).cuda()
    plan = pk.LocalPlan(w.n_obs, w.n_ens, w.n_state, start, ln, pts, tune=True)
    XA = pk.colmajor(len(start), w.n_ens, torch.float32)
    plan.analysis(r, Vd, Dd, XBd, XA)   # first call tunes the configuration
    cfg = plan.sync()
    for _ in range(args.warmup):
        plan.analysis(r, Vd, Dd, XBd, XA)
    ms, ms_med, ms_min = timed_steps(torch, lambda: plan.analysis(r, Vd, Dd, XBd, XA), args.steps)
    plan.sync()
    N = w.n_ens
    # the level iteration of every local solve (6 N^2 n_p) plus its local
    # analysis (2 N^2 n_p + N^2): the work the paper's form would do
    level_flops = float(np.sum(ln)) * 8.0 * N * N + len(ln) * float(N * N)
    xa = XA.cpu().numpy().astype(np.float64)
    # the oracle's own build and local analyses on the same FP32 ensemble
    XB32 = w.XB.astype(np.float32).astype(np.float64)
    V, D = oracle.build_vd(XB32, w.obs_idx, w.y, w.E.astype(np.float32).astype(np.float64))
    ref = oracle.local_analysis(w.r, V, D, XB32, start, ln, pts)
    xb = w.XB.astype(np.float32).astype(np.float64)[pts]
    err = float(np.abs((xa - xb) - (ref - xb)).max() / np.abs(ref - xb).max())
    common = {"avg_launch_us": round(ms * 1e3, 2), "level_iteration_flops": level_flops,
              "level_iteration_TFLOP/s": round(level_flops / (ms * 1e-3) / 1e12, 3),
              "step_ms_median": round(ms_med, 4), "step_ms_min": round(ms_min, 4)}
    if cfg.get("path") == "prefix":
        # FP64 arithmetic the prefix path executes: the chunk sums of both
        # window sums (4 N^2 per ring row), and per problem the N x N LDL^T
        # (N^3 / 3), the two solves (4 N^2), the boundary terms of A_p and
        # Q_p (2 N^2 each) and its edge rows (2 N^2 + 4 N each)
        edge = local_edge_rows(start, ln, w.n_obs)
        flops = (4.0 * N * N * w.n_obs + len(ln) * (N ** 3 / 3.0 + 8.0 * N * N)
                 + float(np.sum(edge)) * (2.0 * N * N + 4.0 * N))
        ach = flops / (ms * 1e-3) / 1e12
        return ms, {"bound": "alu", "achieved": round(ach, 3), "peak": VALU_PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                    "frac": round(ach / VALU_PEAK_TFLOPS["f64"], 4), "traffic": None,
                    "kernel": "local_chunk_kernel + local_scan_kernel + local_prefix_kernel (one graph replay; "
                              "the last is FP64 issue- and latency-bound, one wave per problem)",
                    "alg_flops_per_launch": flops, "edge_rows": int(np.sum(edge)), **common}, cfg, err
    flops = level_flops
    mfma_flops = float(np.sum(ln)) * 2.0 * 64 * 64
    ach = flops / (ms * 1e-3) / 1e12
    return ms, {"bound": "mfma", "achieved": round(ach, 3), "peak": MFMA_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                "frac": round(ach / MFMA_PEAK_TFLOPS["f32"], 4), "traffic": None,
                "kernel": "local_kernel (all local analyses, one graph-replayed launch)",
                "alg_flops_per_launch": flops, "mfma_flops_per_launch": mfma_flops,
                "mfma_TFLOP/s": round(mfma_flops / (ms * 1e-3) / 1e12, 3), **common}, cfg, err


def local_edge_rows(start, ln, n, ch=16):
    """Rows of each window outside its whole 16-row chunks (the rows the
    prefix path takes one by one)."""
    import numpy as np
    nc = -(-n // ch)
    out = np.zeros(len(start), dtype=np.int64)
    for p, (s, m) in enumerate(zip(start, ln)):
        e = s + m
        segs = [(s, min(e, n))] + ([(0, e - n)] if e > n else [])
        for lo, hi in segs:
            c0 = -(-lo // ch)
            c1 = nc if hi == n else hi // ch
            if c0 <= c1:
                out[p] += max(min(c0 * ch, n) - lo, 0) + max(hi - min(c1 * ch, n), 0)
            else:
                out[p] += hi - lo
    return out


def run_loc(w, args, pk, torch):
    """Partial localization (Section 3.1.2) on the Lorenz-96 ring: Z from the
    plain solve, then the localized update with the paper's impact factors
    exp(-d/n_state) on the ring (timed), in FP64 and in FP32."""
    import numpy as np
    import oracle
    out = {}
    ring = length = w.n_state
    loc = torch.as_tensor(w.obs_idx).cuda()
    for storage in ("f64", "f32"):
        tdt = torch.float64 if storage == "f64" else torch.float32
        XB = pk.to_colmajor(w.XB, dtype=tdt)
        E = pk.to_colmajor(w.E, dtype=tdt)
        V, D = pk.enkf_build_vd(XB, loc, torch.as_tensor(w.y).cuda(), E)
        r = torch.as_tensor(w.r).cuda()
        plan = pk.Plan(r, V)
        Z = plan.factor_solve(r, V, D)
        XA = pk.colmajor(w.n_state, w.n_ens, tdt)
        for _ in range(args.warmup):
            plan.localized_analysis(XB, Z, loc, length, -1, ring, XA)
        plan.set_timing(True)
        ms, ms_med, ms_min = timed_steps(torch, lambda: plan.localized_analysis(XB, Z, loc, length, -1, ring, XA),
                                         args.steps)
        t = plan.timing("localize")
        avg_us = t["ms"] * 1e3 / max(t["launches"], 1)
        flops = 4.0 * w.n_state * w.n_obs * w.n_ens
        ach = flops / (avg_us * 1e-6) / 1e12
        # sampled parity: 32 rows (wrapping the ring) against the oracle's formula
        f = (lambda a: a) if storage == "f64" else (lambda a: a.astype(np.float32).astype(np.float64))
        Vh, Zh, XBh = (x.cpu().numpy().astype(np.float64) for x in (V, Z, XB))
        rows = (0, 16)
        ref = oracle.localized_rows(XBh, Vh, Zh, w.obs_idx, length, -1, ring, *rows)
        got = XA[rows[0]:rows[1]].cpu().numpy().astype(np.float64)
        corr = np.abs(ref - XBh[rows[0]:rows[1]]).max()
        err = float(np.abs(got - ref).max() / corr)
        out["localized_" + storage] = {"ms_per_step": round(ms, 4), "ms_median": round(ms_med, 4),
                                       "ms_min": round(ms_min, 4), "analyses_per_s": round(1e3 / ms, 3),
                                       "avg_launch_us": round(avg_us, 2), "alg_flops_per_launch": flops,
                                       "TFLOP/s": round(ach, 2), "sampled_rel_err_vs_oracle": err}
        plan.close()
    return out


CYCLE = {"n_state": 1000, "n_ens": 1000, "cycles": 10, "nsteps": 20, "seed": 20130219}
# (n_state = n_obs, N) across the paper's Lorenz-96 range, timed beside the
# main configuration: a few cycles each, the first one untimed.
CYCLE_SHAPES = [(500, 200), (2000, 800), (5000, 1600)]
CYCLE_SHAPE_CYCLES = 3


def run_cycle(args, pk, torch):
    """The Lorenz-96 cycling filter in the paper's N ~ n_obs regime: n_state =
    n_obs = 1000, N = 1000, R = 0.01^2 I, one time unit (20 RK4 steps) per
    cycle; a step is one cycle (forecast of every member + analysis). Plain
    and blocked solves."""
    import numpy as np
    import synth
    c = CYCLE
    XB0, obs, r, truths, ys, Es = synth.l96_cycle_inputs(c["n_state"], c["n_ens"], c["cycles"], c["nsteps"], c["seed"])
    dev = lambda a: pk.to_colmajor(a) if a.ndim == 2 else torch.as_tensor(a).cuda()
    obs_d, r_d = dev(obs), dev(r)
    ys_d, Es_d = [dev(y) for y in ys], [dev(E) for E in Es]
    out = {}
    for algo in ("plain", "blocked"):
        XB = dev(XB0)
        gen = pk.cycle_l96(XB, obs_d, ys_d, Es_d, r_d, c["nsteps"], algo=algo,
                           block=args.block if algo == "blocked" else 0)
        rf, ra, times = [], [], []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(c["cycles"] + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        k = 0
        for fmean, amean in gen:
            k += 1
            ev[k].record()
            rf.append(fmean)
            ra.append(amean)
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(c["cycles"])]
        steady = ms[min(args.warmup, c["cycles"] - 1):]
        rmse_f = [float(np.sqrt(np.mean((x.cpu().numpy() - truths[i]) ** 2))) for i, x in enumerate(rf)]
        rmse_a = [float(np.sqrt(np.mean((x.cpu().numpy() - truths[i]) ** 2))) for i, x in enumerate(ra)]
        out["cycle_" + algo] = {"ms_per_cycle": round(float(np.mean(steady)), 4),
                                "cycles_per_s": round(1e3 / float(np.mean(steady)), 3),
                                "rmse_forecast": rmse_f, "rmse_analysis": rmse_a}
        print(f"[bench] cycle {algo}: {np.mean(steady):.3f} ms/cycle, RMSE a {rmse_a[-1]:.5f}", file=sys.stderr,
              flush=True)
    if not args.no_cycle_shapes:
        out["cycle_shapes"] = run_cycle_shapes(pk, torch, args.block)
    return out, (XB0, obs, r, truths, ys, Es)


def run_cycle_shapes(pk, torch, block=0):
    """The cycling filter at other (n_state = n_obs, N) shapes of the paper's
    Lorenz-96 range, plain and blocked: milliseconds per cycle over all but the
    first cycle, and the last forecast and analysis RMSE against the truth.
    With N < n_state and no localization the ensemble spans only part of the
    state, so the analysis lowers the error without removing it; the two
    solves agree to roundoff."""
    import numpy as np
    import synth
    c = CYCLE
    res = {}
    for n, N in CYCLE_SHAPES:
        XB0, obs, r, truths, ys, Es = synth.l96_cycle_inputs(n, N, CYCLE_SHAPE_CYCLES, c["nsteps"], c["seed"] + n + N)
        dev = lambda a: pk.to_colmajor(a) if a.ndim == 2 else torch.as_tensor(a).cuda()
        obs_d, r_d = dev(obs), dev(r)
        ys_d, Es_d = [dev(y) for y in ys], [dev(E) for E in Es]
        row = {}
        for algo in ("plain", "blocked"):
            XB = dev(XB0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(CYCLE_SHAPE_CYCLES + 1)]
            torch.cuda.synchronize()
            ev[0].record()
            rf, ra = [], []
            blk = block if algo == "blocked" else 0
            for k, (fmean, amean) in enumerate(pk.cycle_l96(XB, obs_d, ys_d, Es_d, r_d, c["nsteps"], algo=algo,
                                                            block=blk)):
                ev[k + 1].record()
                rf.append(fmean)
                ra.append(amean)
            torch.cuda.synchronize()
            ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(1, CYCLE_SHAPE_CYCLES)]
            rmse = lambda x, t: float(np.sqrt(np.mean((x.cpu().numpy() - t) ** 2)))
            row[algo] = {"ms_per_cycle": round(float(np.mean(ms)), 4),
                         "rmse_forecast": rmse(rf[-1], truths[-1]), "rmse_analysis": rmse(ra[-1], truths[-1])}
            print(f"[bench] cycle n={n} N={N} {algo}: {row[algo]['ms_per_cycle']:.3f} ms/cycle, RMSE f "
                  f"{row[algo]['rmse_forecast']:.5f} a {row[algo]['rmse_analysis']:.5f}", file=sys.stderr, flush=True)
            del XB
        res[f"n{n}_N{N}"] = row
    return res


def run_c5(w, args, pk, torch):
    """c5: N = 1024, n_obs = 524,288, n_state = 2,097,152. The ensemble is kept
    in FP32; the solve runs (a) all-FP32 blocked and (b) FP32 panels refining
    the FP64 system to 1e-10; the analysis update runs on FP32 and on BF16
    matrix cores (FP32 accumulation)."""
    import numpy as np
    f32, f64 = torch.float32, torch.float64
    XB = pk.to_colmajor(w.XB.astype(np.float32), dtype=f32)
    E = pk.to_colmajor(w.E.astype(np.float32), dtype=f32)
    obs = torch.as_tensor(w.obs_idx).cuda()
    y = torch.as_tensor(w.y).cuda()
    r = torch.as_tensor(w.r).cuda()
    n, N = w.n_obs, w.n_ens
    V32, D32 = pk.colmajor(n, N, f32), pk.colmajor(n, N, f32)
    pk.enkf_build_vd(XB, obs, y, E, V32, D32)
    V64, D64 = pk.colmajor(n, N, f64), pk.colmajor(n, N, f64)
    V64.copy_(V32)
    D64.copy_(D32)
    Z32, Z64 = pk.colmajor(n, N, f32), pk.colmajor(n, N, f64)
    XA = pk.colmajor(w.n_state, N, f32)
    res = {}

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        return timed_steps(torch, fn, steps)

    only = [f for f in args.forms.split(",") if f]
    if only:
        # just the analysis product on FP32 / narrow inputs (for profiling):
        # Z from one FP32 blocked solve
        pz = pk.Plan(r, V32, algo="blocked", block=args.block)
        pz.solve(D32, Z32)
        an = {}
        for f in only:
            math = f.replace("analysis_", "")
            ms = timed(lambda: pz.analysis_ex(XB, Z32, XA, math=math), max(2, args.steps))[0]
            an[math] = {"ms": round(ms, 3), "TFLOP/s_incl_VtZ": round(2.0 * w.n_state * N * N / (ms * 1e-3) / 1e12, 2)}
            print(f"[bench] c5 analysis {math}: {ms:.3f} ms", file=sys.stderr, flush=True)
        pz.close()
        return {"analysis_product": an}
    # (a) FP32 blocked, build + factor + solve + analysis (FP32)
    pa = pk.Plan(r, V32, algo="blocked", block=args.block)

    def step_a():
        pk.enkf_build_vd(XB, obs, y, E, V32, D32)
        pa.refactor(r, V32)
        pa.solve(D32, Z32)
        pa.analysis(XB, Z32, XA)
    ms_a, med_a, min_a = timed(step_a, args.steps)
    pa.set_timing(True)
    step_a()
    torch.cuda.synchronize()
    ka = {c: pa.timing(c) for c in CLASSES}
    pa.set_timing(False)
    res["blocked_f32"] = {"ms_per_step": round(ms_a, 3), "ms_median": round(med_a, 3), "ms_min": round(min_a, 3),
                          "solves_per_s": round(1000 / ms_a, 4),
                          "kernels": {c: {"ms": round(v["ms"], 3), "launches": v["launches"],
                                          "TFLOP/s": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] else None}
                                      for c, v in ka.items() if v["launches"]}}
    pa.close()
    # (b) FP32 panels refining the FP64 system, then the FP32 analysis
    pb = pk.Plan(r, V64, algo="blocked", math="f32", block=args.block, refine_max_iter=10, refine_tol=1e-10)
    last = {}

    def step_b():
        pk.enkf_build_vd(XB, obs, y, E, V32, D32)
        V64.copy_(V32)
        D64.copy_(D32)
        pb.refactor(r, V64)
        _, last["info"] = pb.solve(D64, Z64, info=True)
        pb.analysis_ex(XB, Z64, XA, math="f32")
    ms_b, med_b, min_b = timed(step_b, max(1, args.steps))
    pb.set_timing(True)
    step_b()
    torch.cuda.synchronize()
    kb = {c: pb.timing(c) for c in CLASSES}
    pb.set_timing(False)
    res["mixed_f32"] = {"ms_per_step": round(ms_b, 3), "ms_median": round(med_b, 3), "ms_min": round(min_b, 3),
                        "solves_per_s": round(1000 / ms_b, 4),
                        "refine_iters": last["info"]["refine_iters"], "rel_residual": last["info"]["rel_residual"],
                        "kernels": {c: {"ms": round(v["ms"], 3), "launches": v["launches"],
                                        "TFLOP/s": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] else None}
                                    for c, v in kb.items() if v["launches"]}}
    # the analysis product alone, FP32 and BF16 inputs
    an = {}
    for math in ("f32", "bf16"):
        ms = timed(lambda: pb.analysis_ex(XB, Z64, XA, math=math), max(2, args.steps))[0]
        flops = 2.0 * w.n_state * N * N
        an[math] = {"ms": round(ms, 3), "TFLOP/s_incl_VtZ": round(flops / (ms * 1e-3) / 1e12, 2)}
    res["analysis_product"] = an
    pb.close()
    return res


def copy_ms(torch, nbytes):
    """Average time of a plain device copy of nbytes (4 timed after 4 warm-up)."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(4):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 4
    del src, dst
    return ms


def add_measured_peak(roof, dtype, pk, torch):
    """Beside the published peak: the same figure measured on this device (a
    1 GiB device copy for HBM-bound kernels, the MFMA loop of enkf_mfma_peak
    for matrix-core-bound ones) and the kernel's fraction of it."""
    if not isinstance(roof, dict) or roof.get("bound") == "alu":
        return                                    # vector-ALU bound: the published rate only
    if roof.get("unit") == "GB/s":
        nbytes = 1 << 30
        peak = 2 * nbytes / copy_ms(torch, nbytes) / 1e6
        src = "1 GiB device copy, read + write bytes"
    else:
        peak = pk.mfma_peak(dtype)
        src = f"enkf_mfma_peak({dtype})"
    roof["measured_peak"] = round(peak, 1)
    roof["measured_peak_source"] = src
    roof["measured_frac"] = round(roof["achieved"] / peak, 4) if roof.get("achieved") else None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the analysis path is built and timed on a single MI355X; "
              "sharding it across GPUs is not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        ms = copy_ms(torch, nbytes)
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "launches": 8,
                          "copy_ms": round(ms, 4), "copy_GBps_read_plus_write": round(2 * nbytes / ms / 1e6, 1)}),
              flush=True)
        return
    if args.calibrate_mfma:
        import paper_1302_3876_amd as pk
        print(json.dumps({"mfma_TFLOPs_measured": {m: round(pk.mfma_peak(m), 1) for m in ("f64", "f32", "bf16", "f16")},
                          "mfma_TFLOPs_published": MFMA_PEAK_TFLOPS}), flush=True)
        return

    import paper_1302_3876_amd as pk
    import synth

    t0 = time.time()
    if args.workload == "c1":
        w, res = run_c1(args, pk, torch)
        base = None
        if not args.no_cpu_baseline:
            import oracle
            c0, k = time.perf_counter(), 0
            while time.perf_counter() - c0 < 2.0:
                Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
                oracle.analysis(w.XB, Vo, oracle.sm_solve(w.r, Vo, Do)["Z"])
                k += 1
            el = time.perf_counter() - c0
            threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
            base = {"value": round(k / el, 1), "unit": "analyses/s", "cores": threads, "kind": "oracle",
                    "cpu": cpu_model(), "sample": f"{k} whole analysis steps (build + solve + analysis), FP64, "
                                                  f"{el:.2f} s"}
        head = res["graph"]
        out = {"metric": METRIC, "value": head["analyses_per_s"], "unit": "analyses/s", "n_gpus": 1,
               "steps": max(args.steps, 200), "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic (seeded Lorenz-96 truth, ensemble and perturbed observations)",
               "config": {"workload": f"c1: Lorenz-96 n_state={w.n_state}, N={w.n_ens}, every other variable observed "
                                      f"(n_obs={w.n_obs}), R=0.01 I; step = build + plain FP64 factor/solve + analysis, "
                                      f"replayed as one HIP graph (eager launches beside it)", "name": "c1"},
               "roofline": None, "cpu_baseline": base, "forms": res}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "c4":
        w = synth.c4()
        ms, roof, cfg, err = run_local(w, args, pk, torch)
        P = len(w.extra["win_len"])
        base = None
        if not args.no_cpu_baseline:
            import oracle
            import numpy as np
            V, D = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
            c0 = time.perf_counter()
            oracle.local_analysis(w.r, V, D, w.XB, w.extra["win_start"], w.extra["win_len"], w.extra["state_idx"])
            el = time.perf_counter() - c0
            threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
            base = {"value": round(P / el, 2), "unit": "local analyses/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
                    "sample": f"all {P} local analyses of the same workload in FP64 (plain level iteration), {el:.2f} s"}
        out = {"metric": METRIC, "value": round(P / (ms * 1e-3), 1), "unit": "local analyses/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic (seeded Lorenz-96 ring, perturbed observations)",
               "config": {"workload": f"{P} localized analyses on a Lorenz-96 ring n_state={w.n_state}, N={w.n_ens}, "
                                      f"H=I, R=0.01 I, windows n_p~U{{16..512}}; FP32 storage, FP64 pivots; one "
                                      f"graph replay (the path the first call's timing chose)", "name": "c4",
                          "tuned": cfg},
               "roofline": roof, "cpu_baseline": base, "max_increment_err_vs_oracle": err}
        add_measured_peak(out["roofline"], "f32", pk, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "loc":
        w = synth.c6()
        print(f"[bench] loc inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
        res = run_loc(w, args, pk, torch)
        head = res["localized_f64"]
        base = None
        if not args.no_cpu_baseline:
            import oracle
            import numpy as np
            V, D = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
            Zr = oracle.sm_solve(w.r, V, D)["Z"]
            k = 8
            c0 = time.perf_counter()
            oracle.localized_rows(w.XB, V, Zr, w.obs_idx, w.n_state, -1, w.n_state, 0, k)
            el = time.perf_counter() - c0
            threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
            base = {"value": round(k / el / w.n_state, 6), "unit": "localized analyses/s", "cores": threads,
                    "kind": "oracle", "cpu": cpu_model(), "sample": f"{k} of {w.n_state} state rows of the same update in FP64 "
                                                f"({el:.2f} s), scaled to whole analyses"}
        ach = head["TFLOP/s"]
        out = {"metric": METRIC, "value": head["analyses_per_s"], "unit": "localized analyses/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic (seeded Lorenz-96 ensemble, perturbed observations)",
               "config": {"workload": f"partially localized analysis update on a Lorenz-96 ring n_state={w.n_state}, "
                                      f"N={w.n_ens}, every 2nd variable observed (n_obs={w.n_obs}), impact "
                                      f"exp(-d/n_state) on the ring", "name": "loc"},
               "roofline": {"bound": "mfma", "achieved": ach, "peak": MFMA_PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                            "frac": round(ach / MFMA_PEAK_TFLOPS["f64"], 4), "traffic": None,
                            "kernel": "localize64_kernel<double> (resident S tile; S V^T tile, impact weights, times Z)",
                            "avg_launch_us": head["avg_launch_us"], "alg_flops_per_launch": head["alg_flops_per_launch"]},
               "cpu_baseline": base, "forms": res}
        add_measured_peak(out["roofline"], "f64", pk, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "cycle":
        res, inp = run_cycle(args, pk, torch)
        head = res["cycle_blocked"]
        base = None
        if not args.no_cpu_baseline:
            import oracle
            XB0, obs, r, truths, ys, Es = inp
            k = 2
            c0 = time.perf_counter()
            oracle.cycle_l96(XB0, obs, ys[:k], Es[:k], r, CYCLE["nsteps"])
            el = time.perf_counter() - c0
            threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
            base = {"value": round(k / el, 4), "unit": "cycles/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
                    "sample": f"the first {k} cycles of the same run in FP64 ({el:.2f} s)"}
        out = {"metric": METRIC, "value": head["cycles_per_s"], "unit": "cycles/s", "n_gpus": 1,
               "steps": CYCLE["cycles"], "warmup": args.warmup, "ms_per_step": head["ms_per_cycle"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic (seeded Lorenz-96 truth, perturbed observations)",
               "config": {"workload": f"Lorenz-96 cycling filter, n_state = n_obs = {CYCLE['n_state']}, "
                                      f"N = {CYCLE['n_ens']}, R = 0.01^2 I, {CYCLE['nsteps']} RK4 steps per cycle; "
                                      f"blocked solve (plain reported beside it)", "name": "cycle"},
               "roofline": None, "cpu_baseline": base, "forms": res}
        print(json.dumps(out), flush=True)
        return
    if args.workload == "c5":
        w = synth.c5()
        print(f"[bench] c5 inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
        res = run_c5(w, args, pk, torch)
        if "mixed_f32" not in res:
            print(json.dumps({"metric": METRIC, "config": {"name": "c5", "forms": args.forms}, "forms": res}), flush=True)
            return
        head = res["mixed_f32"]
        k = head["kernels"]["gram"]
        ach = k["TFLOP/s"]
        out = {"metric": METRIC, "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32",
               "data": "synthetic (seeded Lorenz-96 ensemble, perturbed observations)",
               "config": {"workload": f"Lorenz-96 ring n_state={w.n_state}, N={w.n_ens}, n_obs={w.n_obs}; FP32 "
                                      f"ensemble; FP32 blocked panels refining the FP64 system to 1e-10; FP32 "
                                      f"analysis product", "name": "c5"},
               "roofline": {"bound": "mfma", "achieved": ach, "peak": MFMA_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                            "frac": round(ach / MFMA_PEAK_TFLOPS["f32"], 4) if ach else None, "traffic": None,
                            "kernel": "tn_partial_kernel<float> (panel products)"},
               "cpu_baseline": None, "forms": res}
        add_measured_peak(out["roofline"], "f32", pk, torch)
        print(json.dumps(out), flush=True)
        return
    w = synth.c2() if args.workload == "c2" else synth.c3()
    print(f"[bench] {args.workload} inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    names = [f for f in args.forms.split(",") if f] or DEFAULT_FORMS[args.workload]
    wnorm = None
    if w.XB is None:
        import oracle   # ||W||_2 estimate of the host-side backward error (a diagnostic)
        wnorm = oracle.norm_w_estimate(w.r, w.V)
    cache = {}
    forms = {}
    for name in names:
        forms[name] = run_form(name, w, args, pk, torch, cache, wnorm)
    cache.clear()
    if args.workload == "c3":
        # headline: the fastest mixed form that meets its residual gate
        mixed = [n for n in names if form_spec(n)[0].startswith("mixed") and forms[n]["gate"]["met"]]
        head = max(mixed, key=lambda n: forms[n]["solves_per_s"]) if mixed else names[0]
    else:
        head = names[0]
    primary = forms[head]
    base = None if args.no_cpu_baseline else cpu_baseline(w, args)
    if args.workload == "c2":
        wl = (f"Lorenz-96 ring n_state={w.n_state}, N={w.n_ens}, n_obs={w.n_obs} (every 4th variable), "
              f"R=diag(U(0.005,0.02)); step = build V,D + factor + solve + analysis update; {head}")
    else:
        wl = (f"c3: n_obs={w.n_obs}, N={w.n_ens}, V_ij = N(0,1) s_i/sqrt(N-1), s_i~U(0.5,2), R=diag(U(0.01,0.1)), "
              f"D~N(0,1); step = factor + solve incl. refinement; {head}: {primary['math']} panels of "
              f"b={primary['block']}, refined in FP64 to relres <= {MIXED_GATE:g}")
    out = {
        "metric": METRIC,
        "value": primary["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": primary["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": primary["storage"],
        "data": "synthetic (seeded; Lorenz-96 ensemble and perturbed observations for c2, direct V/D draws for c3)",
        "config": {"workload": wl, "name": args.workload, "n_state": w.n_state, "n_ens": w.n_ens, "n_obs": w.n_obs,
                   "form": head, "block": primary["block"], "math": primary["math"]},
        "roofline": roofline_of(primary, head),
        "cpu_baseline": base,
        "rel_residual": primary["rel_residual"],
        "backward_error": primary["backward_error"],
        "forms": forms,
    }
    # speedups only between forms that meet their accuracy gates
    ok = {k: v for k, v in forms.items() if v["gate"]["met"]}
    if "plain_f64" in ok:
        p = ok["plain_f64"]["ms_per_step"]
        out["speedup_vs_plain_f64_at_gate"] = {k: round(p / v["ms_per_step"], 3) for k, v in ok.items()}
    if "blocked_f64" in ok:
        p = ok["blocked_f64"]["ms_per_step"]
        out["speedup_vs_blocked_f64_at_gate"] = {k: round(p / v["ms_per_step"], 3) for k, v in ok.items()}
    if ok:
        best = max(ok, key=lambda k: ok[k]["solves_per_s"])
        out["fastest_form_at_gate"] = {"form": best, "solves_per_s": ok[best]["solves_per_s"],
                                       "rel_residual": ok[best]["rel_residual"],
                                       "backward_error": ok[best]["backward_error"]}
    add_measured_peak(out["roofline"], out["roofline"].get("peak_type", primary["math"])
                      if out["roofline"]["unit"] != "GB/s" else "f64", pk, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
