"""Pins of the two diagnostics every FP64 parity gate leans on: the estimate
of ||W||_2 (max r + the largest eigenvalue of V^T V) and the normwise
backward error eta = ||D - W Z||_F / (||W||_2 ||Z||_F + ||D||_F), each
against the explicit W = R + V V^T (Section 3, eq. system-to-solve) formed
on small inputs and its spectral norm from a dense SVD.

Both R and V V^T are positive semidefinite, so Weyl's inequality gives
max(max r, sigma_max(V)^2) <= ||W||_2 <= max r + sigma_max(V)^2: the
estimate lies in [||W||_2, 2 ||W||_2], and equals ||W||_2 when R is a
multiple of I and V has rank one (W = c I + v v^T, ||W||_2 = c + ||v||^2).
An estimate that inflated ||W||_2 beyond this factor would loosen every
gate that divides by it; the planted variants below must fail these pins."""
import numpy as np
import pytest

import oracle
import synth


def _explicit_w(r, V):
    return np.diag(r) + V @ V.T


def _cases():
    g = np.random.default_rng(2024)
    out = []
    for n, N, rs, vs in [(60, 5, (0.5, 2.0), 1.0), (80, 12, (0.01, 0.1), 1.0), (50, 4, (1.0, 3.0), 1e-3),
                         (40, 40, (0.2, 0.2), 3.0), (30, 45, (0.005, 0.02), 0.5)]:
        r = g.uniform(*rs, n) if rs[0] != rs[1] else np.full(n, rs[0])
        V = g.standard_normal((n, N)) * vs / np.sqrt(N)
        D = g.standard_normal((n, 3))
        out.append((r, V, D))
    return out


@pytest.mark.parametrize("case", range(5))
def test_norm_w_estimate_within_weyl_bounds(case):
    r, V, _ = _cases()[case]
    w2 = np.linalg.norm(_explicit_w(r, V), 2)
    est = oracle.norm_w_estimate(r, V)
    assert w2 * (1 - 1e-12) <= est <= 2.0 * w2 * (1 + 1e-12), (est, w2)


@pytest.mark.parametrize("n,c", [(25, 0.3), (64, 2.0)])
def test_norm_w_estimate_exact_for_rank_one(n, c):
    v = synth.normal(31, 1, n)[:, None]
    r = np.full(n, c)
    est = oracle.norm_w_estimate(r, v)
    closed = c + float(v[:, 0] @ v[:, 0])
    assert abs(est - closed) <= 1e-13 * closed
    assert abs(np.linalg.norm(_explicit_w(r, v), 2) - closed) <= 1e-12 * closed


def test_norm_w_estimate_tight_when_one_term_dominates():
    # V negligible: ||W|| = max r; R negligible: ||W|| = sigma_max(V)^2
    g = np.random.default_rng(7)
    r = g.uniform(1.0, 4.0, 40)
    V = g.standard_normal((40, 6)) * 1e-9
    assert abs(oracle.norm_w_estimate(r, V) - r.max()) <= 1e-12 * r.max()
    V = g.standard_normal((40, 6)) * 1e4
    r = np.full(40, 1e-9)
    w2 = np.linalg.norm(_explicit_w(r, V), 2)
    assert abs(oracle.norm_w_estimate(r, V) - w2) <= 1e-10 * w2


@pytest.mark.parametrize("case", range(5))
def test_backward_error_matches_definition(case):
    """eta from the oracle against its definition with the explicit W: with
    the estimate in [||W||, 2||W||], eta lies in [eta_true / 2, eta_true];
    for a perturbed solution of known residual the numerator is exact."""
    r, V, D = _cases()[case]
    W = _explicit_w(r, V)
    Z = np.linalg.solve(W, D)
    Zp = Z + 1e-6 * np.random.default_rng(case).standard_normal(Z.shape)
    rho = D - W @ Zp
    eta_true = np.linalg.norm(rho) / (np.linalg.norm(W, 2) * np.linalg.norm(Zp) + np.linalg.norm(D))
    eta = oracle.backward_error(r, V, Zp, D)
    assert 0.5 * eta_true * (1 - 1e-9) <= eta <= eta_true * (1 + 1e-9), (eta, eta_true)
    assert abs(np.linalg.norm(oracle.residual(r, V, Zp, D)) - np.linalg.norm(rho)) <= 1e-9 * np.linalg.norm(rho)


def test_backward_error_exact_for_rank_one():
    n, c = 50, 0.7
    v = synth.normal(32, 1, n)[:, None]
    r = np.full(n, c)
    D = synth.normal(33, 1, n * 2).reshape(n, 2)
    W = _explicit_w(r, v)
    Zp = np.linalg.solve(W, D) + 1e-5
    rho = D - W @ Zp
    eta_true = np.linalg.norm(rho) / ((c + float(v[:, 0] @ v[:, 0])) * np.linalg.norm(Zp) + np.linalg.norm(D))
    assert abs(oracle.backward_error(r, v, Zp, D) - eta_true) <= 1e-9 * eta_true


# Planted mistakes in the estimate (each a plausible slip) must break a pin.
def _mut_trace(r, V):
    return float(np.max(r) + np.sum(V * V))             # ||V||_F^2 instead of sigma_max^2


def _mut_min_r(r, V):
    g = V.T @ V
    return float(np.min(r) + np.max(np.linalg.eigvalsh(g)))


def _mut_sqrt(r, V):
    g = V.T @ V
    return float(np.max(r) + np.sqrt(np.max(np.linalg.eigvalsh(g))))


@pytest.mark.parametrize("mutant", [_mut_trace, _mut_min_r, _mut_sqrt])
def test_planted_estimate_mistakes_fail(mutant, monkeypatch):
    monkeypatch.setattr(oracle, "norm_w_estimate", mutant)
    failed = 0
    for case in range(5):
        r, V, _ = _cases()[case]
        w2 = np.linalg.norm(_explicit_w(r, V), 2)
        est = oracle.norm_w_estimate(r, V)
        if not (w2 * (1 - 1e-12) <= est <= 2.0 * w2 * (1 + 1e-12)):
            failed += 1
    for n, c in [(25, 0.3), (64, 2.0)]:
        v = synth.normal(31, 1, n)[:, None]
        closed = c + float(v[:, 0] @ v[:, 0])
        if abs(oracle.norm_w_estimate(np.full(n, c), v) - closed) > 1e-13 * closed:
            failed += 1
    assert failed > 0
