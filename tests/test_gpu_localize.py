"""Partial localization (Section 3.1.2) on the fused HIP kernel against the
FP64 oracle's formula, through the C ABI.

Tolerances: the correction sums N products over the state members and n_obs
weighted products over the observations; in FP64 the difference from the
oracle's order is a few units of roundoff of the absolute sums, so it is
bounded by 1e-12 times the largest |correction| (plus the X^B scale for the
addition). FP32 storage and FP32 matrix cores: 2e-5 of the same scale."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


def _inputs(n_state, N, stride, seed):
    """Lorenz-96-shaped ensemble on a ring, every `stride`-th point observed,
    V from the anomalies, Z from an FP64 solve of the same system."""
    g = np.random.default_rng(seed)
    XB = 2.3 + 3.6 * g.standard_normal((n_state, N))
    loc = np.arange(0, n_state, stride, dtype=np.int64)
    n_obs = loc.shape[0]
    A = (XB - XB.mean(axis=1, keepdims=True)) / np.sqrt(N - 1)
    V = A[loc]
    r = g.uniform(0.5, 1.5, n_obs)
    D = g.standard_normal((n_obs, N))
    Z = oracle.sm_solve(r, V, D)["Z"]
    return XB, V, Z, loc, r


def _gate(XA, ref, XB, tol):
    corr = np.max(np.abs(ref - XB))
    err = np.max(np.abs(XA - ref))
    assert err <= tol * (corr + 1e-3 * np.max(np.abs(XB))), (err, corr)


@pytest.mark.parametrize("n_state,N,stride,length,radius,ring", [
    (512, 40, 2, 512.0, -1, 512),      # the paper's Lorenz-96 form: ring, length = n_state
    (100, 160, 3, 7.5, 10, 0),         # N > 128 (two column chunks), radius, no ring, ragged tiles
    (2048, 64, 2, 64.0, -1, 2048),
    (33, 2, 1, 3.0, 4, 33),
])
def test_localized_fp64_matches_oracle(n_state, N, stride, length, radius, ring):
    import torch
    print(f"localize fp64 n_state={n_state} N={N} stride={stride}", flush=True)
    pk = _pk()
    XB, V, Z, loc, r = _inputs(n_state, N, stride, seed=n_state + N)
    plan = pk.Plan(dev(r), dev(V))
    XA = plan.localized_analysis(dev(XB), dev(Z), dev(loc), length, radius, ring)
    torch.cuda.synchronize()
    ref = oracle.localized_analysis(XB, V, Z, loc, length, radius, ring)
    _gate(host(XA), ref, XB, 1e-12)


def test_localized_without_taper_is_the_analysis():
    import torch
    pk = _pk()
    XB, V, Z, loc, r = _inputs(300, 24, 2, seed=9)
    plan = pk.Plan(dev(r), dev(V))
    XA = host(plan.localized_analysis(dev(XB), dev(Z), dev(loc), 1e300))
    torch.cuda.synchronize()
    _gate(XA, oracle.analysis(XB, V, Z), XB, 1e-12)


@pytest.mark.parametrize("n_state,N,stride,radius", [
    (1024, 48, 2, -1),     # members padded to 64 (resident S tile)
    (257, 64, 3, 40),      # ragged row tile and observation step, radius
    (300, 96, 2, -1),      # N > 64: the general kernel
])
def test_localized_fp32(n_state, N, stride, radius):
    import torch
    print(f"localize fp32 n_state={n_state} N={N} stride={stride}", flush=True)
    pk = _pk()
    XB, V, Z, loc, r = _inputs(n_state, N, stride, seed=5 + N)
    f = lambda a: a.astype(np.float32).astype(np.float64)
    plan = pk.Plan(dev(r), dev(V, torch.float32))
    L = float(n_state)
    XA = plan.localized_analysis(dev(XB, torch.float32), dev(Z, torch.float32), dev(loc), L, radius, n_state)
    torch.cuda.synchronize()
    ref = oracle.localized_analysis(f(XB), f(V), f(Z), loc, L, radius, n_state)
    _gate(host(XA), ref, f(XB), 2e-5)


def test_localized_bad_arguments():
    import torch
    pk = _pk()
    XB, V, Z, loc, r = _inputs(64, 8, 2, seed=1)
    plan = pk.Plan(dev(r), dev(V))
    for kw in ({"length": 0.0}, {"length": float("inf")}, {"length": 1.0, "ring": 10}):
        with pytest.raises(pk.EnkfError) as e:
            plan.localized_analysis(dev(XB), dev(Z), dev(loc), **kw)
        assert e.value.code == 1


@pytest.mark.slow
def test_localized_full_size_sampled_rows():
    """The loc workload at full size (Lorenz-96 ring n_state = 32,768, N = 64,
    n_obs = 16,384, impact exp(-d/n_state) on the ring) in FP64, in the
    launch bench.py times: three blocks of 64 state rows (the first, one in
    the middle, the last, i.e. both ends of the ring) against the oracle's
    rows, same bound as the small cases."""
    import torch
    import synth as sy
    print("localize full size, sampled rows", flush=True)
    pk = _pk()
    w = sy.c6()
    XBd = dev(w.XB)
    V, D = pk.enkf_build_vd(XBd, dev(w.obs_idx), dev(w.y), dev(w.E))
    plan = pk.Plan(dev(w.r), V)
    Z = plan.solve(D)
    ring = length = w.n_state
    XA = host(plan.localized_analysis(XBd, Z, dev(w.obs_idx), length, -1, ring))
    torch.cuda.synchronize()
    Vh, Zh = host(V), host(Z)
    for r0 in (0, w.n_state // 2 - 32, w.n_state - 64):
        ref = oracle.localized_rows(w.XB, Vh, Zh, w.obs_idx, length, -1, ring, r0, r0 + 64)
        _gate(XA[r0:r0 + 64], ref, w.XB[r0:r0 + 64], 1e-12)
