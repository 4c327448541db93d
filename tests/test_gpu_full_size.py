"""The blocked and mixed-precision solves at the full size of workload c3
(n = 2,097,152 observations, N = 256), in the configuration bench.py times
(panels of 128 levels), through the C ABI.

At this size the oracle cannot solve the whole system in a test's time, so
the checks are (1) the backward error of the device's Z in FP64,
||D - R Z - V (V^T Z)|| / ||D||, formed on the host with numpy (a property
that holds at any size: the paper's method solves (R + V V^T) Z = D), and
(2) outputs the oracle computes one by one: the pivots gamma_0..gamma_7 of
the first eight levels depend only on the first eight columns of V, so the
oracle's level iteration on those columns gives them exactly.

Bounds: blocked FP64 without refinement reaches ~1.5e-11 here (the panel
Woodbury products lose a few digits to the conditioning of M), so 1e-10;
the mixed FP32 form refines until the FP64 residual is <= 1e-10 (the gate it
is run with). Pivots: FP64 panels, rtol 1e-10; FP32 panels with FP64
pivots, rtol 1e-5 (the FP32 Gram products)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def c3():
    return synth.c3()


def _relres(w, Z):
    rho = w.D - w.r[:, None] * Z - w.V @ (w.V.T @ Z)
    return float(np.linalg.norm(rho) / np.linalg.norm(w.D))


def _first_gammas(w, k=8):
    return oracle.sm_solve(w.r, np.ascontiguousarray(w.V[:, :k]), np.ascontiguousarray(w.D[:, :1]))["gamma"]


@pytest.mark.parametrize("math,rtol", [("f64", 1e-10), ("f32", 1e-5)])
def test_c3_full_size(c3, math, rtol):
    import torch
    import paper_1302_3876_amd as pk
    print(f"c3 full size, blocked, panels {math}", flush=True)
    w = c3
    if math == "f64":
        plan = pk.Plan(dev(w.r), dev(w.V), algo="blocked", block=128)
    else:
        plan = pk.Plan(dev(w.r), dev(w.V), algo="blocked", math="f32", block=128, refine_max_iter=8,
                       refine_tol=1e-10)
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    g, _ = plan.pivots()
    Zh = host(Z)
    del Z
    plan.close()
    rr = _relres(w, Zh)
    print({"rel_residual": rr, "info": info}, flush=True)
    assert rr <= 1e-10
    assert np.allclose(g[:8], _first_gammas(w), rtol=rtol, atol=0)


def test_c5_ensemble_shape():
    """The c5 configuration (N = 1024 members in FP32, panels of 128 levels,
    FP32 panels refining the FP64 system to 1e-10, the FP32 analysis product
    with K = N = 1024) on a Lorenz-96 ring of 65,536 variables (n_obs =
    16,384): build against the oracle, backward error and first pivots of the
    solve, and the analysis on 256 sampled state rows against the oracle's
    update of those rows (FP32 storage and products: 2e-5 of the largest
    increment)."""
    import torch
    import paper_1302_3876_amd as pk
    print("c5 shape, n_state=65536, N=1024", flush=True)
    w = synth.c5(n_state=65536)
    XB32 = w.XB.astype(np.float32).astype(np.float64)
    E32 = w.E.astype(np.float32).astype(np.float64)
    f32 = torch.float32
    XBd = pk.to_colmajor(XB32, dtype=f32)
    n, N = w.n_obs, w.n_ens
    V32, D32 = pk.colmajor(n, N, f32), pk.colmajor(n, N, f32)
    pk.enkf_build_vd(XBd, dev(w.obs_idx), dev(w.y), pk.to_colmajor(E32, dtype=f32), V32, D32)
    Vo, Do = oracle.build_vd(XB32, w.obs_idx, w.y, E32)
    V, D = host(V32), host(D32)
    assert np.max(np.abs(V - Vo)) <= 4 * 2.0 ** -24 * np.max(np.abs(Vo)) + 4 * N * 2.0 ** -52 * np.max(np.abs(XB32))
    assert np.max(np.abs(D - Do)) <= 4 * 2.0 ** -24 * np.max(np.abs(Do))
    plan = pk.Plan(dev(w.r), dev(V), algo="blocked", math="f32", block=128, refine_max_iter=10, refine_tol=1e-10)
    Z, info = plan.solve(dev(D), info=True)
    XA = host(plan.analysis_ex(XBd, Z, math="f32"))
    torch.cuda.synchronize()
    g, _ = plan.pivots()
    Zh = host(Z)
    plan.close()
    rho = D - w.r[:, None] * Zh - V @ (V.T @ Zh)
    rr = float(np.linalg.norm(rho) / np.linalg.norm(D))
    print({"rel_residual": rr, "info": info}, flush=True)
    assert rr <= 1e-10
    g8 = oracle.sm_solve(w.r, np.ascontiguousarray(V[:, :8]), np.ascontiguousarray(D[:, :1]))["gamma"]
    assert np.allclose(g[:8], g8, rtol=1e-5, atol=0)
    rows = np.random.default_rng(5).choice(w.n_state, 256, replace=False)
    ref = oracle.analysis(XB32[rows], V, Zh)
    inc, inco = XA[rows] - XB32[rows], ref - XB32[rows]
    assert np.max(np.abs(inc - inco)) <= 2e-5 * np.max(np.abs(inco))


def test_c5_full_size_sampled():
    """The c5 configuration at its full size (n_state = 2,097,152, N = 1024,
    n_obs = 524,288; FP32 ensemble) in the launch configuration bench.py
    times (panels of 128 levels, FP32 panels refining the FP64 system to
    1e-10, the FP32 analysis product), checked on samples: the build on 512
    observation rows against the oracle; the solve by its FP64 residual on
    32 columns (formed on the host with numpy) and its first eight pivots
    against the oracle's level iteration on V's first columns; the analysis
    increment on 256 state rows against S_rows (V^T Z) with the N x N factor
    formed on the host in FP64 (a plain matrix product: the oracle's own
    loops would need minutes for it). Bounds: build and pivots as in the
    smaller c5 test; sampled residual 1e-9 (the device's whole-matrix gate is
    1e-10); increment 2e-5 of its largest entry (FP32 storage and products)."""
    import torch
    import paper_1302_3876_amd as pk
    print("c5 full size", flush=True)
    w = synth.c5()
    n, N = w.n_obs, w.n_ens
    f32 = torch.float32
    g = np.random.default_rng(55)
    XBd = pk.to_colmajor(w.XB.astype(np.float32), dtype=f32)
    Ed = pk.to_colmajor(w.E.astype(np.float32), dtype=f32)
    V32, D32 = pk.colmajor(n, N, f32), pk.colmajor(n, N, f32)
    pk.enkf_build_vd(XBd, dev(w.obs_idx), dev(w.y), Ed, V32, D32)
    torch.cuda.synchronize()
    V, D = host(V32), host(D32)
    orows = np.sort(g.choice(n, 512, replace=False))
    XBs = w.XB[w.obs_idx[orows]].astype(np.float32).astype(np.float64)
    Es = w.E[orows].astype(np.float32).astype(np.float64)
    Vo, Do = oracle.build_vd(XBs, np.arange(len(orows), dtype=np.int64), w.y[orows], Es)
    assert np.max(np.abs(V[orows] - Vo)) <= 4 * 2.0 ** -24 * np.max(np.abs(Vo)) + 4 * N * 2.0 ** -52 * np.max(np.abs(XBs))
    assert np.max(np.abs(D[orows] - Do)) <= 4 * 2.0 ** -24 * np.max(np.abs(Do))
    del Ed, XBs, Es
    plan = pk.Plan(dev(w.r), dev(V), algo="blocked", math="f32", block=128, refine_max_iter=10, refine_tol=1e-10)
    Z, info = plan.solve(dev(D), info=True)
    XA = plan.analysis_ex(XBd, Z, math="f32")
    torch.cuda.synchronize()
    gam, _ = plan.pivots()
    Zh = host(Z)
    del Z
    plan.close()
    print({"info": info}, flush=True)
    assert info["rel_residual"] <= 1e-10
    cols = np.sort(g.choice(N, 32, replace=False))
    Zc = Zh[:, cols]
    rho = D[:, cols] - w.r[:, None] * Zc - V @ (V.T @ Zc)
    rr = float(np.linalg.norm(rho) / np.linalg.norm(D[:, cols]))
    print({"sampled_rel_residual": rr}, flush=True)
    assert rr <= 1e-9
    g8 = oracle.sm_solve(w.r, np.ascontiguousarray(V[:, :8]), np.ascontiguousarray(D[:, :1]))["gamma"]
    assert np.allclose(gam[:8], g8, rtol=1e-5, atol=0)
    G = V.T @ Zh / np.sqrt(N - 1)
    del Zh, V, D
    srows = np.sort(g.choice(w.n_state, 256, replace=False))
    XBr = w.XB[srows].astype(np.float32).astype(np.float64)
    ref = (XBr - XBr.mean(axis=1, keepdims=True)) @ G
    inc = host(XA[torch.as_tensor(srows, device=XA.device)]) - XBr
    err = float(np.max(np.abs(inc - ref)))
    print({"increment_err": err, "scale": float(np.max(np.abs(ref)))}, flush=True)
    assert err <= 2e-5 * np.max(np.abs(ref))
