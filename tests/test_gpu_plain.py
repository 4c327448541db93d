"""Parity of the plain HIP path (build, level sweeps, analysis) with the FP64
oracle, on the same seeded inputs, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, fp64_gate, host, rel

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


# 600,007 (odd: one row per load) and 600,008 rows give more row tiles than
# the grid's row blocks, so each block walks several tiles; 2,100,007 and
# 2,100,008 rows pass 2048 row tiles (512 row blocks), and their 18 columns
# exceed the last-level cache (the streamed, non-temporal layout);
# 2,097,147 (2^21 - 5) and 4,194,301 (2^22 - 3) rows give exactly 512 row
# blocks (one and two streamed tiles each, ragged last tile), so the
# streamed levels run their row blocks in chunks of 256
# (64, 32, 48) fills the single-block path's 56 KiB of LDS exactly
# (n (2N + nrhs) doubles); (65, 32, 48) is one row past it; 1024 rows is its
# row limit, 1025 one past
@pytest.mark.parametrize("n,N,nrhs", [(1, 1, 1), (5, 3, 2), (7, 1, 3), (1000, 17, 17), (4099, 33, 5),
                                      (16384, 96, 96), (70001, 40, 40), (3, 50, 50), (600007, 9, 9),
                                      (600008, 9, 5), (2100007, 9, 9), (2100008, 9, 9), (64, 32, 48),
                                      (65, 32, 48), (20, 20, 20), (200, 7, 1),
                                      (1024, 2, 1), (1025, 2, 1), (2097147, 9, 9), (4194301, 5, 5)])
def test_solve_fp64_matches_oracle(n, N, nrhs):
    import torch
    print(f"solve fp64 n={n} N={N} nrhs={nrhs}", flush=True)
    r, V, D = synth.small_vd(n, N, seed=1000 + n + N, nrhs=nrhs)
    plan = _pk().Plan(dev(r), dev(V), max_nrhs=nrhs)
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    ref = oracle.sm_solve(r, V, D)
    fp64_gate(r, V, D, host(Z), ref["Z"])
    g, _ = plan.pivots()
    assert np.allclose(g, ref["gamma"], rtol=1e-12, atol=0)
    assert info["device_status"] == 0


@pytest.mark.parametrize("n,N", [(4099, 33), (65536, 64), (1100004, 8)])
def test_solve_fp32_matches_oracle(n, N):
    import torch
    print(f"solve fp32 n={n} N={N}", flush=True)
    r, V, D = synth.small_vd(n, N, seed=2000 + n, r_range=(0.005, 0.02), v_scale=0.3)
    plan = _pk().Plan(dev(r), dev(V, torch.float32))
    Z = plan.solve(dev(D, torch.float32))
    torch.cuda.synchronize()
    ref = oracle.sm_solve(r, V.astype(np.float32).astype(np.float64), D.astype(np.float32).astype(np.float64))
    # FP32 storage: every level rounds the updated columns to FP32 (unit
    # roundoff 6e-8); the forward error stays within a few hundred units times
    # the growth in the pivots.
    assert rel(host(Z), ref["Z"]) < 1e-4


@pytest.mark.parametrize("n,N,nrhs", [(1, 1, 1), (5, 3, 2), (4099, 33, 5), (16384, 96, 96), (70001, 40, 40),
                                      (3, 50, 50), (1002, 7, 11), (600008, 9, 9), (2100008, 9, 9), (64, 32, 48),
                                      (65, 32, 48), (20, 20, 20)])
def test_fused_factor_solve_matches_oracle_and_split_path(n, N, nrhs):
    """One level loop over [U, Z] (enkf_sm_factor_solve): parity with the
    oracle, and bitwise the same Z and pivots as refactor + solve (every
    column's products are summed in the same order in both)."""
    import torch
    print(f"fused fp64 n={n} N={N} nrhs={nrhs}", flush=True)
    pk = _pk()
    r, V, D = synth.small_vd(n, N, seed=3000 + n + N, nrhs=nrhs)
    rd, Vd, Dd = dev(r), dev(V), dev(D)
    plan = pk.Plan(rd, Vd, max_nrhs=max(nrhs, N))
    Zs = plan.solve(Dd)
    gs, _ = plan.pivots()
    Zf, info = plan.factor_solve(rd, Vd, Dd, info=True)
    torch.cuda.synchronize()
    gf, _ = plan.pivots()
    assert info["device_status"] == 0
    assert np.array_equal(host(Zf), host(Zs))
    assert np.array_equal(gf, gs)
    fp64_gate(r, V, D, host(Zf), oracle.sm_solve(r, V, D)["Z"])
    # the factor it leaves serves later solves
    assert np.array_equal(host(plan.solve(Dd)), host(Zs))


def test_fused_factor_solve_fp32_alias_and_zero_rhs():
    import torch
    pk = _pk()
    n, N = 65536, 64
    r, V, D = synth.small_vd(n, N, seed=77, r_range=(0.005, 0.02), v_scale=0.3)
    rd, Vd = dev(r), dev(V, torch.float32)
    plan = pk.Plan(rd, Vd)
    Zs = host(plan.solve(dev(D, torch.float32)))
    Dd = dev(D, torch.float32)
    Zf = plan.factor_solve(rd, Vd, Dd, Dd)    # Z aliases D
    torch.cuda.synchronize()
    assert np.array_equal(host(Zf), Zs)
    empty = pk.colmajor(n, 0, torch.float32)
    plan.factor_solve(rd, Vd, empty, empty)   # factorisation only
    assert np.array_equal(host(plan.solve(dev(D, torch.float32))), Zs)


@pytest.mark.parametrize("n", [1001, 101])     # 101: the single-block path (Z aliases D in its LDS copy)
def test_unaligned_leading_dimension_and_alias(n):
    import torch
    pk = _pk()
    N = 9
    r, V, D = synth.small_vd(n, N, seed=5)
    Vp = pk.colmajor(n + 1, N)[:n]           # ld = n + 1 (odd): scalar path
    Vp.copy_(torch.as_tensor(V))
    Dp = pk.colmajor(n + 3, N)[:n]
    Dp.copy_(torch.as_tensor(D))
    plan = pk.Plan(dev(r), Vp)
    Z = plan.solve(Dp, Dp)                    # in place: Z aliases D
    torch.cuda.synchronize()
    fp64_gate(r, V, D, host(Z), oracle.sm_solve(r, V, D)["Z"])


def test_zero_rhs_and_zero_column():
    import torch
    pk = _pk()
    n, N = 300, 6
    r, V, D = synth.small_vd(n, N, seed=9)
    V[:, 2] = 0.0
    plan = pk.Plan(dev(r), dev(V))
    empty = pk.colmajor(n, 0)
    plan.solve(empty, empty)
    Z = plan.solve(dev(D))
    torch.cuda.synchronize()
    g, _ = plan.pivots()
    assert g[2] == 1.0
    fp64_gate(r, V, D, host(Z), oracle.sm_solve(r, V, D)["Z"])


def test_nonpositive_r_is_reported():
    pk = _pk()
    n, N = 200, 4
    r, V, D = synth.small_vd(n, N, seed=3)
    r[17] = 0.0
    plan = pk.Plan(dev(r), dev(V))
    with pytest.raises(pk.EnkfError) as e:
        plan.info()
    assert e.value.code == 2


def test_bitwise_reproducible():
    import torch
    pk = _pk()
    r, V, D = synth.small_vd(50000, 24, seed=12)
    a = host(pk.Plan(dev(r), dev(V)).solve(dev(D)))
    b = host(pk.Plan(dev(r), dev(V)).solve(dev(D)))
    torch.cuda.synchronize()
    assert np.array_equal(a, b)


def _full_path(w, dtype):
    import torch
    pk = _pk()
    XB = dev(w.XB, dtype)
    E = dev(w.E, dtype)
    V, D = pk.enkf_build_vd(XB, dev(w.obs_idx), dev(w.y), E)
    plan = pk.Plan(dev(w.r), V)
    Z = plan.solve(D)
    XA = plan.analysis(XB, Z)
    torch.cuda.synchronize()
    return host(V), host(D), host(Z), host(XA), plan


def test_c1_full_path_fp64():
    w = synth.c1()
    V, D, Z, XA, plan = _full_path(w, None)
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    # the member mean is a sum of N FP64 terms in an order the definition does
    # not fix: the two orders differ by at most ~N eps max|X^B|
    N, eps = w.XB.shape[1], 2.0 ** -52
    assert np.max(np.abs(V - Vo)) <= 4 * N * eps * np.max(np.abs(w.XB)) / np.sqrt(N - 1)
    assert np.max(np.abs(D - Do)) <= 4 * eps * (np.max(np.abs(w.y)) + np.max(np.abs(w.E)) + np.max(np.abs(w.XB)))
    Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
    fp64_gate(w.r, Vo, Do, Z, Zo)
    XAo = oracle.analysis(w.XB, Vo, Zo)
    assert rel(XA - w.XB, XAo - w.XB) < 1e-11


@pytest.mark.slow
def test_c2_full_path_fp64_full_size():
    print("c2 full size fp64", flush=True)
    w = synth.c2()
    V, D, Z, XA, plan = _full_path(w, None)
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    assert rel(V, Vo) < 1e-14 and rel(D, Do) < 1e-15
    Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
    g = fp64_gate(w.r, Vo, Do, Z, Zo)
    print(g, flush=True)
    # the blocked form on the same inputs (one panel of 96 levels), without
    # refinement: the panel applies M^{-1} through its LDL^T factor
    import torch
    pk = _pk()
    bplan = pk.Plan(dev(w.r), dev(Vo), algo="blocked")
    Zb = host(bplan.solve(dev(Do)))
    torch.cuda.synchronize()
    gb = fp64_gate(w.r, Vo, Do, Zb, Zo)
    print({"blocked": gb}, flush=True)
    # every element of the increment, not only the norm. Here the oracle's
    # own rounding dominates: its ascending FP64 sums over 262,144
    # observations leave a relative residual of 7e-11 (the device's is
    # ~7e-13), and on the host its increment differs from that of an
    # LDL^T-blocked solve (relative residual 4e-12) by 1.5e-10 of the largest
    # increment; bound: ten times the larger of the two relative residuals
    XAo = oracle.analysis(w.XB, Vo, Zo)
    inc, inco = XA - w.XB, XAo - w.XB
    einc = np.max(np.abs(inc - inco)) / np.max(np.abs(inco))
    bound = 10.0 * max(g["relres_gpu"], g["relres_oracle"])
    print({"increment_max_rel": einc, "bound": bound}, flush=True)
    assert einc <= bound


@pytest.mark.slow
def test_c2_full_path_fp32_full_size():
    import torch
    print("c2 full size fp32", flush=True)
    w = synth.c2()
    V, D, Z, XA, plan = _full_path(w, torch.float32)
    XB32 = w.XB.astype(np.float32).astype(np.float64)
    E32 = w.E.astype(np.float32).astype(np.float64)
    Vo, Do = oracle.build_vd(XB32, w.obs_idx, w.y, E32)
    Zo = oracle.sm_solve(w.r, Vo, Do)["Z"]
    rz = rel(Z, Zo)
    XAo = oracle.analysis(XB32, Vo, Zo)
    ra = rel(XA - XB32, XAo - XB32)
    # FP32 storage and arithmetic: forward error up to kappa(W) times the
    # FP32 rounding unit (2^-24)
    kappa = oracle.norm_w_estimate(w.r, Vo) / float(np.min(w.r))
    bound = kappa * 2.0 ** -24
    print({"z_rel": rz, "increment_rel": ra, "kappa": kappa, "bound": bound}, flush=True)
    assert rz < bound and ra < bound
