"""Block-diagonal R (Section 2.1; Step 1 block by block) on the HIP path,
plain and blocked algorithms, FP64 and FP32 storage, against the FP64
oracle's block-R solve through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


def _case(sizes, N, nrhs, seed, vscale=0.7):
    g = np.random.default_rng(seed)
    blocks = []
    for s in sizes:
        A = g.standard_normal((s, s))
        blocks.append(A @ A.T / s + np.diag(g.uniform(0.2, 1.0, s)))
    n = int(sum(sizes))
    V = g.standard_normal((n, N)) * vscale / np.sqrt(max(N - 1, 1))
    D = g.standard_normal((n, nrhs))
    return blocks, V, D


def _dense_w(blocks, V):
    import scipy.linalg as sla
    return sla.block_diag(*blocks) + V @ V.T


def _plan(pk, blocks, V, algo="plain", dtype=None, **kw):
    import torch
    off, packed = oracle.pack_blocks(blocks)
    Vd = dev(V, dtype or torch.float64)
    return pk.Plan(None, Vd, algo=algo, block_r=(off, torch.as_tensor(packed).cuda()), **kw), Vd


def _sizes(n_blocks, lo, hi, seed):
    return list(np.random.default_rng(seed).integers(lo, hi + 1, n_blocks))


@pytest.mark.parametrize("algo,sizes,N,nrhs", [
    ("plain", [3, 1, 4, 2, 5], 4, 2),
    ("plain", None, 33, 33),          # 2000 blocks of 1..8 rows
    ("plain", [64] * 40, 16, 5),      # the largest blocks
    ("blocked", None, 48, 48),
    ("blocked", [17] * 30 + [1], 20, 7),
])
def test_block_r_matches_oracle(algo, sizes, N, nrhs):
    import torch
    pk = _pk()
    if sizes is None:
        sizes = _sizes(2000, 1, 8, seed=N)
    print(f"block R {algo} blocks={len(sizes)} n={sum(sizes)} N={N}", flush=True)
    blocks, V, D = _case(sizes, N, nrhs, seed=len(sizes) + N)
    plan, _ = _plan(pk, blocks, V, algo=algo, max_nrhs=max(N, nrhs))
    Z, info = plan.solve(dev(D), info=True)
    torch.cuda.synchronize()
    assert info["device_status"] == 0
    ref = oracle.sm_solve_block_r(blocks, V, D)
    Zh = host(Z)
    W = _dense_w(blocks, V) if sum(sizes) <= 3000 else None
    # backward error against the explicit W (FP64 bound), forward vs the oracle
    if W is not None:
        eta = np.linalg.norm(W @ Zh - D) / (np.linalg.norm(W, 2) * np.linalg.norm(Zh) + np.linalg.norm(D))
        assert eta <= 1e-12, eta
    assert np.linalg.norm(Zh - ref["Z"]) <= 1e-10 * np.linalg.norm(ref["Z"])
    g, _ = plan.pivots()
    assert np.allclose(g, ref["gamma"], rtol=1e-10, atol=0)


def test_block_r_fp32_and_refactor():
    import torch
    pk = _pk()
    sizes = _sizes(3000, 1, 12, seed=3)
    blocks, V, D = _case(sizes, 24, 24, seed=4)
    plan, Vd = _plan(pk, blocks, V, dtype=torch.float32)
    f = lambda a: a.astype(np.float32).astype(np.float64)
    Z = host(plan.solve(dev(D, torch.float32)))
    torch.cuda.synchronize()
    ref = oracle.sm_solve_block_r(blocks, f(V), f(D))["Z"]
    assert np.linalg.norm(Z - ref) <= 1e-4 * np.linalg.norm(ref)
    # refactor with scaled blocks: R -> 2R
    blocks2 = [2.0 * b for b in blocks]
    _, packed2 = oracle.pack_blocks(blocks2)
    plan.refactor_block_r(torch.as_tensor(packed2).cuda(), Vd)
    Z2 = host(plan.solve(dev(D, torch.float32)))
    torch.cuda.synchronize()
    ref2 = oracle.sm_solve_block_r(blocks2, f(V), f(D))["Z"]
    assert np.linalg.norm(Z2 - ref2) <= 1e-4 * np.linalg.norm(ref2)


def test_block_r_not_spd_and_unsupported():
    import torch
    pk = _pk()
    blocks, V, D = _case([3, 3, 3], 4, 1, seed=9)
    blocks[1] = -blocks[1]
    plan, _ = _plan(pk, blocks, V)
    with pytest.raises(pk.EnkfError) as e:
        plan.info()
    assert e.value.code == 2
    blocks, V, D = _case([3, 3], 4, 1, seed=10)
    for algo, kw in (("plain", {"pivot": True}), ("blocked", {"math": "f32", "refine_max_iter": 2})):
        with pytest.raises(pk.EnkfError) as e:
            _plan(pk, blocks, V, algo=algo, **kw)
        assert e.value.code == 6
    with pytest.raises(pk.EnkfError) as e:
        _plan(pk, [np.eye(65)], np.zeros((65, 2)))
    assert e.value.code == 6
