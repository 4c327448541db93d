"""Parity of the blocked and mixed-precision HIP paths with the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, fp64_gate, host, rel

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


@pytest.mark.parametrize("n,N,b,nrhs", [(64, 1, 1, 1), (1000, 17, 5, 17), (4099, 33, 8, 7), (16384, 96, 32, 96),
                                        (16384, 96, 96, 96), (70001, 40, 40, 40), (3, 50, 16, 50),
                                        (9000, 130, 64, 130), (5000, 128, 128, 16), (3001, 127, 127, 5),
                                        (2000, 101, 101, 9)])
def test_blocked_fp64_matches_oracle(n, N, b, nrhs):
    import torch
    print(f"blocked fp64 n={n} N={N} b={b} nrhs={nrhs}", flush=True)
    r, V, D = synth.small_vd(n, N, seed=3000 + n + N + b, nrhs=nrhs)
    plan = _pk().Plan(dev(r), dev(V), algo="blocked", block=b, max_nrhs=nrhs)
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    ref = oracle.sm_solve(r, V, D)
    fp64_gate(r, V, D, host(Z), ref["Z"])
    g, _ = plan.pivots()
    # the LDL^T pivots of each panel are the gammas of its levels
    assert np.allclose(g, ref["gamma"], rtol=1e-10, atol=0)


@pytest.mark.parametrize("n,N,b", [(4099, 33, 16), (65536, 64, 64)])
def test_blocked_fp32_matches_oracle(n, N, b):
    import torch
    r, V, D = synth.small_vd(n, N, seed=4000 + n, r_range=(0.005, 0.02), v_scale=0.3)
    plan = _pk().Plan(dev(r), dev(V, torch.float32), algo="blocked", block=b)
    Z = plan.solve(dev(D, torch.float32))
    torch.cuda.synchronize()
    ref = oracle.sm_solve(r, V.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64))
    assert rel(host(Z), ref["Z"]) < 1e-4


@pytest.mark.parametrize("n,N,b", [(20000, 32, 16), (131072, 64, 32)])
def test_mixed_f32_refines_to_fp64_accuracy(n, N, b):
    import torch
    print(f"mixed f32 n={n} N={N} b={b}", flush=True)
    w = synth.direct_vd_workload("c3-small", n, N, seed=5000 + n)
    plan = _pk().Plan(dev(w.r), dev(w.V), algo="blocked", math="f32", block=b, refine_max_iter=6,
                      refine_tol=1e-11)
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    print(info, flush=True)
    assert info["refine_iters"] >= 1 and info["rel_residual"] <= 1e-11
    ref = oracle.sm_solve(w.r, w.V, w.D)
    fp64_gate(w.r, w.V, w.D, host(Z), ref["Z"])


def test_blocked_analysis_matches_plain():
    import torch
    pk = _pk()
    w = synth.c2(n_state=65536, n_ens=48)
    XB = dev(w.XB)
    V, D = pk.enkf_build_vd(XB, dev(w.obs_idx), dev(w.y), dev(w.E))
    plan = pk.Plan(dev(w.r), V, algo="blocked", block=16)
    Z = plan.solve(D)
    XA = plan.analysis(XB, Z)
    torch.cuda.synchronize()
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
    fp64_gate(w.r, Vo, Do, host(Z), Zo)
    XAo = oracle.analysis(w.XB, Vo, Zo)
    assert rel(host(XA) - w.XB, XAo - w.XB) < 1e-9


def test_refactor_reuses_plan():
    import torch
    pk = _pk()
    r1, V1, D1 = synth.small_vd(5000, 20, seed=1)
    r2, V2, D2 = synth.small_vd(5000, 20, seed=2)
    for algo in ("plain", "blocked"):
        plan = pk.Plan(dev(r1), dev(V1), algo=algo, block=8 if algo == "blocked" else 0)
        r2d, V2d = dev(r2), dev(V2)
        plan.refactor(r2d, V2d)
        Z = plan.solve(dev(D2))
        torch.cuda.synchronize()
        fp64_gate(r2, V2, D2, host(Z), oracle.sm_solve(r2, V2, D2)["Z"])


@pytest.mark.parametrize("math", ["f32", "bf16", "f16", "bf16x3", "f16x2"])
def test_mixed_every_math_well_conditioned(math):
    # pivots gamma ~ 15: the one-pass 16-bit forms converge only where the
    # pivots times the input rounding (bf16 4e-3, f16 5e-4) stay well below 1
    import torch
    n, N = 1000, 16
    r, V, D = synth.small_vd(n, N, seed=77, r_range=(0.5, 2.0), v_scale=0.5)
    plan = _pk().Plan(dev(r), dev(V), algo="blocked", math=math, block=16, refine_max_iter=12, refine_tol=1e-12)
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    print(math, info, flush=True)
    assert info["rel_residual"] <= 1e-12
    fp64_gate(r, V, D, host(Z), oracle.sm_solve(r, V, D)["Z"])


@pytest.mark.parametrize("math,maxit", [("bf16x3", 30), ("f16x2", 8), ("f32", 8)])
def test_mixed_split_forms_reach_gate_on_c3_like_data(math, maxit):
    """The split forms on c3-distributed data refine to the mixed gate,
    judged by the host's FP64 residual of the returned Z (the host's own
    evaluation error is ~2e-12 of ||D|| on this data, measured against an
    80-bit evaluation). The device's report is printed, not gated: the
    refinement drives the device's own FP64 residual to its stopping
    tolerance, so that report sits at or below the true residual."""
    import torch
    n, N, b = 131072, 64, 32
    w = synth.direct_vd_workload("c3-small", n, N, seed=6000)
    plan = _pk().Plan(dev(w.r), dev(w.V), algo="blocked", math=math, block=b, refine_max_iter=maxit,
                      refine_tol=1e-10)
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    rr = oracle.rel_residual(w.r, w.V, host(Z), w.D)
    print(math, info, "host relres", rr, flush=True)
    assert rr <= 1e-10
    assert info["rel_residual"] <= 1e-10


@pytest.mark.parametrize("math", ["f32", "bf16x3"])
@pytest.mark.parametrize("n,N", [(131149, 64), (40077, 160)])
def test_mixed_device_residual_norm(math, n, N):
    """||rho|| / ||D|| as the device forms it (the squares of rho summed in the
    residual product's epilogue, per block then in a fixed order; ||D||^2 once
    per solve) against the host's FP64 residual of the returned Z. Taken after
    the first low-precision solve alone (no refinement step), where rho is
    far above the rounding of its own evaluation. The row counts leave padding
    blocks in the grid (their partials must be zero); N = 160 takes the
    128 x 64 tiles with three column tiles."""
    import torch
    w = synth.direct_vd_workload("c3-small", n, N, seed=6001)
    plan = _pk().Plan(dev(w.r), dev(w.V), algo="blocked", math=math, block=32, refine_max_iter=0, refine_tol=0.0)
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    Zh = host(Z)
    rho = w.D - w.r[:, None] * Zh - w.V @ (w.V.T @ Zh)
    rr = np.linalg.norm(rho) / np.linalg.norm(w.D)
    print(math, n, N, info, rr, flush=True)
    assert info["refine_iters"] == 0
    assert abs(info["rel_residual"] - rr) <= 1e-6 * rr


@pytest.mark.parametrize("math,tol", [("f32", 2e-5), ("bf16x3", 2e-5), ("f16x2", 2e-5), ("bf16", 2e-2), ("f16", 5e-3)])
def test_analysis_ex_fp32_ensemble(math, tol):
    """The analysis update on an FP32 ensemble with FP32/narrow matrix-core
    inputs, against the FP64 oracle on the same (FP32-rounded) ensemble."""
    import torch
    pk = _pk()
    w = synth.c2(n_state=131072, n_ens=96)
    XB32 = w.XB.astype(np.float32).astype(np.float64)
    E32 = w.E.astype(np.float32).astype(np.float64)
    Vo, Do = oracle.build_vd(XB32, w.obs_idx, w.y, E32)
    plan = pk.Plan(dev(w.r), dev(Vo), algo="blocked")
    Z = plan.solve(dev(Do))
    XA = plan.analysis_ex(dev(XB32, torch.float32), Z, math=math)
    torch.cuda.synchronize()
    XAo = oracle.analysis(XB32, Vo, oracle.sm_solve(w.r, Vo, Do)["Z"])
    err = rel(host(XA) - XB32, XAo - XB32)
    print(math, err, flush=True)
    assert err < tol


def test_blocked_fp64_refinement_restores_accuracy():
    """FP64 panels with FP64 refinement (F64/F64 and refine_max_iter > 0) on
    an ill-conditioned system (R = 1e-4 I, large ensemble spread, the
    capacitance matrix has condition ~1e5). The panel update applies M^{-1}
    through its LDL^T factor (two triangular products), so the unrefined
    solve already reaches the oracle's residual level; two residual
    corrections keep it there."""
    import torch
    import paper_1302_3876_amd as pk
    n, N = 20000, 96
    g = np.random.default_rng(11)
    V = g.standard_normal((n, N)) * 0.4 / np.sqrt(N - 1)
    r = np.full(n, 1e-4)
    D = g.standard_normal((n, N)) * 0.4
    ref = oracle.sm_solve(r, V, D)
    rr_or = oracle.rel_residual(r, V, ref["Z"], D)
    plain = pk.Plan(dev(r), dev(V), algo="blocked")
    Z0 = host(plain.solve(dev(D)))
    # a fixed number of steps (tol 0): the residual's own FP64 evaluation
    # floor here is ~1e-11, so a tolerance below it would never be met
    plan = pk.Plan(dev(r), dev(V), algo="blocked", refine_max_iter=2, refine_tol=0.0)
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    rr0 = oracle.rel_residual(r, V, Z0, D)
    rr = oracle.rel_residual(r, V, host(Z), D)
    print({"unrefined": rr0, "refined": rr, "oracle": rr_or}, flush=True)
    assert info["refine_iters"] == 2
    assert rr <= max(1e-12, 2.0 * rr_or), (rr, rr_or, rr0)
    assert rr0 <= max(1e-12, 2.0 * rr_or), (rr, rr_or, rr0)


def test_mixed_solve_latches_bad_r():
    """The mixed form applies R^{-1} while narrowing D and each residual
    (Step 1 fused into that copy); a non-positive r_i seen there latches
    NOT_SPD like the separate Step 1 does. The plan borrows r, so r is spoiled
    on the device after the (valid) factorization."""
    import torch
    pk = _pk()
    n, N = 1000, 16
    r, V, D = synth.small_vd(n, N, seed=78)
    rd = dev(r)
    plan = pk.Plan(rd, dev(V), algo="blocked", math="f32", block=16, refine_max_iter=2, refine_tol=1e-12)
    torch.cuda.synchronize()
    rd[5] = -1.0
    with pytest.raises(pk.EnkfError) as e:
        plan.solve(dev(D), info=True)
    assert e.value.code == 2
    plan.close()


@pytest.mark.parametrize("math,refine", [("f32", 2), ("f64", 1), ("bf16x3", 3)])
def test_refined_solves_reject_overlapping_rhs(math, refine):
    """Refined and mixed solves read D again for every residual after Z has
    been written, so any overlap of Z with D is refused on the host (in place,
    or shifted by a column); the out-of-place solve still matches the oracle."""
    import torch
    pk = _pk()
    n, N = 2000, 16
    r, V, D = synth.small_vd(n, N, seed=80)
    rd, Vd = dev(r), dev(V)
    plan = pk.Plan(rd, Vd, algo="blocked", math=math, block=8, refine_max_iter=refine, refine_tol=0.0)
    Dd = dev(D)
    for call in (lambda: plan.solve(Dd, Dd), lambda: plan.factor_solve(rd, Vd, Dd, Dd)):
        with pytest.raises(pk.EnkfError) as e:
            call()
        assert e.value.code == 1
    big = pk.colmajor(n, N + 1)
    big[:, :N].copy_(torch.as_tensor(D))
    with pytest.raises(pk.EnkfError) as e:
        plan.solve(big[:, :N], big[:, 1:])
    assert e.value.code == 1
    Z, info = plan.solve(Dd, info=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(Dd), D)
    fp64_gate(r, V, D, host(Z), oracle.sm_solve(r, V, D)["Z"])


def test_unrefined_solves_reject_partial_overlap():
    """The plain and the unrefined blocked solves run in place (Z == D), but
    a Z that overlaps D otherwise is refused."""
    import torch
    pk = _pk()
    n, N = 1500, 12
    r, V, D = synth.small_vd(n, N, seed=82)
    for algo in ("plain", "blocked"):
        plan = pk.Plan(dev(r), dev(V), algo=algo, block=4 if algo == "blocked" else 0)
        big = pk.colmajor(n, N + 1)
        big[:, :N].copy_(torch.as_tensor(D))
        with pytest.raises(pk.EnkfError) as e:
            plan.solve(big[:, :N], big[:, 1:])
        assert e.value.code == 1
        Dd = dev(D)
        Z = plan.solve(Dd, Dd)
        torch.cuda.synchronize()
        fp64_gate(r, V, D, host(Z), oracle.sm_solve(r, V, D)["Z"])


@pytest.mark.parametrize("math", ["f16", "f16x2"])
def test_fp16_forms_scale_large_right_hand_sides(math):
    """The well-conditioned system of test_mixed_every_math_well_conditioned
    with R and V V^T both scaled by 1e-6 (the same pivots): R^{-1} D is then
    ~1e6, beyond the FP16 range (65504). The FP16 forms divide each
    right-hand side by the rms of R^{-1} times it before narrowing, so the
    solve converges to the same accuracy instead of overflowing."""
    import torch
    n, N = 1000, 16
    r, V, D = synth.small_vd(n, N, seed=77, r_range=(0.5, 2.0), v_scale=0.5)
    r, V = r * 1e-6, V * 1e-3
    plan = _pk().Plan(dev(r), dev(V), algo="blocked", math=math, block=16, refine_max_iter=12, refine_tol=1e-12)
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    Zh = host(Z)
    print(math, info, flush=True)
    assert np.all(np.isfinite(Zh))
    assert oracle.rel_residual(r, V, Zh, D) <= 1e-12
    fp64_gate(r, V, D, Zh, oracle.sm_solve(r, V, D)["Z"])


@pytest.mark.parametrize("algo,math,refine", [("plain", "f64", 0), ("blocked", "f64", 0), ("blocked", "f64", 1),
                                              ("blocked", "f32", 4), ("blocked", "f32", 0)])
def test_diagnose_flag_reports_backward_error(algo, math, refine):
    """ENKF_FLAG_DIAGNOSE: every synchronous solve reports the relative
    residual and eta = ||D - W Z|| / (||W||_2 ||Z|| + ||D||) of its Z.
    (1) The device's ||W||_2 estimate (max r + the Rayleigh quotient of V^T V
    after 60 power steps), recovered from the two reports, against the
    oracle's (max r + the largest eigenvalue of the Gram): within 2%.
    (2) Where the residual is far above the rounding of its evaluation (the
    unrefined FP32-panel solve, ~1e-6) the reports match the host's FP64
    values of the returned Z to 1e-6. (3) Where it is at the rounding floor
    (FP64 forms, ~1e-13) both evaluations are mostly rounding: the device
    report stays below twice the host's plus 1e-13. An in-place solve and a
    plan without the flag report -1."""
    import torch
    pk = _pk()
    w = synth.c2(n_state=65536, n_ens=48)
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    plan = pk.Plan(dev(w.r), dev(Vo), algo=algo, math=math, block=16 if algo == "blocked" else 0,
                   refine_max_iter=refine, refine_tol=0.0, diagnose=True)
    Z, info = plan.solve(dev(Do), info=True)
    torch.cuda.synchronize()
    Zh = host(Z)
    rr = oracle.rel_residual(w.r, Vo, Zh, Do)
    eta = oracle.backward_error(w.r, Vo, Zh, Do)
    dn, zn = np.linalg.norm(Do), np.linalg.norm(Zh)
    w_dev = (info["rel_residual"] * dn / info["backward_error"] - dn) / zn
    w_or = oracle.norm_w_estimate(w.r, Vo)
    print(algo, math, refine, info, {"relres": rr, "eta": eta, "w_dev": w_dev, "w_oracle": w_or}, flush=True)
    assert info["backward_error"] > 0 and info["rel_residual"] > 0 and info["hip_error"] == 0
    assert abs(w_dev - w_or) <= 0.02 * w_or
    if math == "f32" and refine == 0:
        assert rr > 1e-8
        assert abs(info["rel_residual"] - rr) <= 1e-6 * rr
        assert abs(info["backward_error"] - eta) <= 0.02 * eta
    else:
        assert info["rel_residual"] <= 2.0 * rr + 1e-13
        assert info["backward_error"] <= 1e-15
    if algo == "plain":
        Dd = dev(Do)
        _, info2 = plan.solve(Dd, Dd, info=True)
        assert info2["backward_error"] == -1.0
    plan.close()
    plain = pk.Plan(dev(w.r), dev(Vo))
    _, info3 = plain.solve(dev(Do), info=True)
    assert info3["backward_error"] == -1.0 and info3["rel_residual"] == -1.0


@pytest.mark.parametrize("math", ["f64", "f32"])
def test_autotuned_panel_width(math):
    """ENKF_FLAG_AUTOTUNE with block 0: init times each candidate width (32,
    64, 96, 128 up to N) on the plan's data and keeps the fastest; the solve
    with it matches the oracle; a second plan of the same shape reuses the
    width without timing again."""
    import torch
    pk = _pk()
    n, N = 40000, 100
    w = synth.direct_vd_workload("c3-small", n, N, seed=6100)
    kw = dict(algo="blocked", math=math, autotune=True)
    if math != "f64":
        kw.update(refine_max_iter=8, refine_tol=1e-11)
    plan = pk.Plan(dev(w.r), dev(w.V), **kw)
    tun = plan.tuning()
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    print(math, tun, info, flush=True)
    assert sorted(tun) == [32, 64, 96] and all(v > 0 for v in tun.values())
    assert info["block"] == min(tun, key=tun.get)
    fp64_gate(w.r, w.V, w.D, host(Z), oracle.sm_solve(w.r, w.V, w.D)["Z"])
    plan2 = pk.Plan(dev(w.r), dev(w.V), **kw)
    assert plan2.tuning() == {} and plan2.info()["block"] == info["block"]
