"""The analysis update X^A = X^B + S V^T Z (Section 3.1, the SMEnKF update)
through the C ABI, against the FP64 oracle, over ensemble sizes that take
each of the analysis kernels: the small-N kernel (N <= 96 in FP64, <= 128
in FP32; member padding to 32, 64, 96 and 128) and the general tiled kernel
beyond, with row counts that leave a ragged last row tile.

Tolerances: FP64 — the increment is a sum of N products of FP64 values
whose order differs from the oracle's, so every element of it agrees to a
few units of roundoff of the largest increment (1e-11 of it). FP32 storage
and FP32 matrix cores — 2e-5 of the largest increment (the FP32 rounding of
X^B, G and the products, summed over N <= 160 terms)."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


def _inputs(n_state, n_obs, N, seed):
    g = np.random.default_rng(seed)
    XB = 1.7 + 2.9 * g.standard_normal((n_state, N))
    V = g.standard_normal((n_obs, N)) / np.sqrt(N - 1)
    Z = g.standard_normal((n_obs, N))
    r = g.uniform(0.5, 1.5, n_obs)
    return XB, V, Z, r


def _check(XA, XB, ref, tol):
    inc, inco = XA - XB, ref - XB
    err = np.max(np.abs(inc - inco))
    assert err <= tol * np.max(np.abs(inco)), (err, np.max(np.abs(inco)))


@pytest.mark.parametrize("n_state,N", [(1000, 2), (777, 33), (4096, 64), (300, 65), (2113, 96), (513, 97), (200, 160)])
def test_analysis_fp64(n_state, N):
    import torch
    print(f"analysis fp64 n_state={n_state} N={N}", flush=True)
    pk = _pk()
    XB, V, Z, r = _inputs(n_state, 257, N, seed=n_state + N)
    plan = pk.Plan(dev(r), dev(V))
    XA = host(plan.analysis(dev(XB), dev(Z)))
    torch.cuda.synchronize()
    _check(XA, XB, oracle.analysis(XB, V, Z), 1e-11)


@pytest.mark.parametrize("n_state,N", [(1000, 20), (640, 64), (2113, 96), (1029, 128), (300, 129)])
def test_analysis_fp32_storage(n_state, N):
    import torch
    print(f"analysis fp32 n_state={n_state} N={N}", flush=True)
    pk = _pk()
    XB, V, Z, r = _inputs(n_state, 193, N, seed=7 * N + n_state)
    XB32 = XB.astype(np.float32).astype(np.float64)
    plan = pk.Plan(dev(r), dev(V))
    XA = host(plan.analysis_ex(dev(XB32, torch.float32), dev(Z), math="f32"))
    torch.cuda.synchronize()
    _check(XA, XB32, oracle.analysis(XB32, V, Z), 2e-5)


@pytest.mark.parametrize("n_state,n_obs,N", [(4096, 100, 16), (4097, 100, 16), (256, 20, 64), (300, 50, 8),
                                             (40, 20, 20)])
def test_analysis_fp64_small_systems(n_state, n_obs, N):
    """Few observations and members (the c1 shape among them), ragged state
    row counts; a second call on the same plan gives the same result."""
    import torch
    print(f"analysis fp64 small n_state={n_state} n_obs={n_obs} N={N}", flush=True)
    pk = _pk()
    XB, V, Z, r = _inputs(n_state, n_obs, N, seed=n_state + 3 * N)
    plan = pk.Plan(dev(r), dev(V))
    ref = oracle.analysis(XB, V, Z)
    XA = host(plan.analysis(dev(XB), dev(Z)))
    XA2 = host(plan.analysis(dev(XB), dev(Z)))
    torch.cuda.synchronize()
    _check(XA, XB, ref, 1e-11)
    assert np.array_equal(XA, XA2)


def test_analysis_in_place_output_and_reuse():
    """A second call on other data gives that data's update (the persistent
    kernel keeps no state between calls)."""
    import torch
    pk = _pk()
    XB, V, Z, r = _inputs(1500, 129, 96, seed=3)
    plan = pk.Plan(dev(r), dev(V))
    XA1 = host(plan.analysis(dev(XB), dev(Z)))
    XB2 = XB[::-1].copy()
    XA2 = host(plan.analysis(dev(XB2), dev(Z)))
    torch.cuda.synchronize()
    _check(XA1, XB, oracle.analysis(XB, V, Z), 1e-11)
    _check(XA2, XB2, oracle.analysis(XB2, V, Z), 1e-11)


@pytest.mark.parametrize("prec,math,N,tol", [("f64", "f64", 160, 1e-11), ("f32", "f32", 256, 2e-5),
                                             ("f32", "bf16x3", 256, 2e-5)])
def test_analysis_many_row_tiles(prec, math, N, tol):
    """Enough rows (more than 2048 row tiles) that one block walks all column
    tiles of its row tile; 512 sampled rows against the oracle's update of
    those rows."""
    import torch
    print(f"analysis many row tiles {prec}/{math} N={N}", flush=True)
    pk = _pk()
    n_state = 2048 * 128 + 77
    XB, V, Z, r = _inputs(n_state, 301, N, seed=N + 11)
    if prec == "f32":
        XB = XB.astype(np.float32).astype(np.float64)
    plan = pk.Plan(dev(r), dev(V))
    if prec == "f64":
        XA = host(plan.analysis(dev(XB), dev(Z)))
    else:
        XA = host(plan.analysis_ex(dev(XB, torch.float32), dev(Z), math=math))
    torch.cuda.synchronize()
    rows = np.concatenate([np.arange(64), np.random.default_rng(N).choice(n_state, 384, replace=False),
                           np.arange(n_state - 64, n_state)])
    _check(XA[rows], XB[rows], oracle.analysis(XB[rows], V, Z), tol)


@pytest.mark.parametrize("math,n_state,N", [("bf16", 131072, 1024), ("bf16", 65536 + 37, 1000), ("f16", 70001, 96),
                                            ("bf16", 65600, 20)])
def test_analysis_16bit_resident_tile(math, n_state, N):
    """The analysis product on one-pass 16-bit inputs with many state rows
    (the kernel that keeps each 64-row tile of the centred ensemble in the
    LDS for all output columns): against the FP64 oracle's update of the same
    FP32 ensemble on 512 sampled rows (both ends of a ragged last tile
    included) and over all rows by the increment norm. Inputs rounded to
    16 bits: 2e-2 (BF16) / 5e-3 (FP16) of the largest increment."""
    import torch
    pk = _pk()
    print(f"analysis {math} n_state={n_state} N={N}", flush=True)
    g = np.random.default_rng(n_state + N)
    n_obs = 4096
    XB32 = (8.0 + g.standard_normal((n_state, N))).astype(np.float32).astype(np.float64)
    V = np.asfortranarray(g.standard_normal((n_obs, N)) * 0.05)
    V -= V.mean(axis=1, keepdims=True)
    Z = np.asfortranarray(g.standard_normal((n_obs, N)))
    r = np.full(n_obs, 1.0)
    plan = pk.Plan(dev(r), dev(V, torch.float32), algo="blocked")
    XA = host(plan.analysis_ex(dev(XB32, torch.float32), dev(Z, torch.float32), math=math))
    torch.cuda.synchronize()
    V32 = V.astype(np.float32).astype(np.float64)
    Z32 = Z.astype(np.float32).astype(np.float64)
    rows = np.unique(np.concatenate([g.choice(n_state, 500, replace=False), np.arange(6), n_state - 1 - np.arange(6)]))
    ref = oracle.analysis(XB32[rows], V32, Z32)
    inc, inco = XA[rows] - XB32[rows], ref - XB32[rows]
    err = float(np.max(np.abs(inc - inco)) / np.max(np.abs(inco)))
    tol = 2e-2 if math == "bf16" else 5e-3
    print({"max_err": err}, flush=True)
    assert err < tol
    assert np.all(np.isfinite(XA))
