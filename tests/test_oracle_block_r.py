"""Pins of the block-diagonal-R oracle (R = diag(R_1..R_B) of Section 2.1,
Step 1 block by block): a dense Cholesky solve of the explicit
W = R + V V^T, the diagonal case (1 x 1 blocks) against the diagonal
oracle, one dense block, the determinant lemma for the pivots, and a
non-SPD block reported."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle


def _blocks(sizes, seed):
    g = np.random.default_rng(seed)
    out = []
    for s in sizes:
        A = g.standard_normal((s, s))
        out.append(A @ A.T / s + np.diag(g.uniform(0.2, 1.0, s)))
    return out


def _case(sizes, N, nrhs, seed):
    g = np.random.default_rng(seed + 1)
    n = sum(sizes)
    return _blocks(sizes, seed), g.standard_normal((n, N)) * 0.7, g.standard_normal((n, nrhs))


@pytest.mark.parametrize("sizes,N", [([3, 1, 4, 2, 5], 4), ([8] * 6, 7), ([1] * 9 + [6], 3), ([30], 5)])
def test_matches_dense_cholesky(sizes, N):
    blocks, V, D = _case(sizes, N, 3, seed=len(sizes) + N)
    W = sla.block_diag(*blocks) + V @ V.T
    ref = sla.solve(W, D, assume_a="pos")
    Z = oracle.sm_solve_block_r(blocks, V, D)["Z"]
    assert np.linalg.norm(Z - ref) <= 1e-12 * np.linalg.norm(ref)


def test_unit_blocks_equal_diagonal_oracle():
    g = np.random.default_rng(3)
    n, N = 40, 6
    r = g.uniform(0.5, 2.0, n)
    V, D = g.standard_normal((n, N)), g.standard_normal((n, N))
    a = oracle.sm_solve_block_r([np.array([[x]]) for x in r], V, D)
    b = oracle.sm_solve(r, V, D)
    assert np.allclose(a["Z"], b["Z"], rtol=1e-13, atol=1e-15)
    assert np.allclose(a["gamma"], b["gamma"], rtol=1e-13, atol=0)


def test_pivots_product_is_the_determinant_ratio():
    # prod gamma_k = det(I + V^T R^{-1} V) = det(R + V V^T) / det(R)
    blocks, V, D = _case([4, 3, 5], 5, 1, seed=8)
    R = sla.block_diag(*blocks)
    g = oracle.sm_solve_block_r(blocks, V, D)["gamma"]
    _, ld_w = np.linalg.slogdet(R + V @ V.T)
    _, ld_r = np.linalg.slogdet(R)
    assert np.isclose(np.sum(np.log(g)), ld_w - ld_r, rtol=1e-12, atol=1e-12)


def test_non_spd_block_is_reported():
    blocks, V, D = _case([3, 3], 2, 1, seed=2)
    blocks[1] = -blocks[1]
    with pytest.raises(oracle.OracleError) as e:
        oracle.sm_solve_block_r(blocks, V, D)
    assert e.value.code == 2
