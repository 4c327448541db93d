"""Pins for the FP64 oracle: each check ties it to something other than itself
(a dense factorisation, exact rational arithmetic, the paper's recursive
definition, theorems and closed forms, the paper's operation counts).

Runs on the CPU only."""
import os
import shutil
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _problem(n, N, seed, nrhs=None, r_range=(0.5, 2.0), v_scale=1.0):
    return synth.small_vd(n, N, seed, r_range=r_range, v_scale=v_scale, nrhs=nrhs)


def _dense_solve(r, V, D):
    W = np.diag(r) + V @ V.T
    return sla.cho_solve(sla.cho_factor(W, lower=True), D)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# --- the whole solve against a dense Cholesky factorisation of W ------------
@pytest.mark.parametrize("n,N,nrhs", [(1, 1, 1), (1, 5, 5), (5, 1, 1), (30, 8, 8), (8, 30, 30),
                                      (200, 32, 32), (64, 64, 64), (50, 10, 3), (40, 6, 0)])
def test_matches_dense_cholesky(n, N, nrhs):
    r, V, D = _problem(n, N, seed=100 + n * 7 + N, nrhs=nrhs)
    out = oracle.sm_solve(r, V, D)
    if nrhs == 0:
        assert out["Z"].shape == (n, 0)
        return
    Zref = _dense_solve(r, V, D)
    assert _rel(out["Z"], Zref) < 1e-12


def test_matches_dense_wide_r_range():
    # r spanning 1e-6..1e6: still a well-posed SPD system.
    n, N = 60, 12
    r, V, D = _problem(n, N, seed=7)
    r = 10.0 ** np.linspace(-6, 6, n)
    out = oracle.sm_solve(r, V, D)
    Zref = _dense_solve(r, V, D)
    # cond(W) ~ 3e10 here: the relative residual is conditioning-limited, the
    # normwise backward error is not.
    assert oracle.backward_error(r, V, out["Z"], D) < 1e-16
    assert _rel(out["Z"], Zref) < 1e-10


# --- exact rational arithmetic on a tiny system ------------------------------
def _exact_solve(W, D):
    n = len(W)
    A = [[Fraction(W[i][j]) for j in range(n)] + [Fraction(D[i][k]) for k in range(len(D[0]))] for i in range(n)]
    m = len(A[0])
    for c in range(n):
        p = next(i for i in range(c, n) if A[i][c] != 0)
        A[c], A[p] = A[p], A[c]
        for i in range(n):
            if i != c and A[i][c] != 0:
                f = A[i][c] / A[c][c]
                A[i] = [A[i][j] - f * A[c][j] for j in range(m)]
    return [[A[i][n + k] / A[i][i] for k in range(m - n)] for i in range(n)]


def test_exact_rational_tiny():
    rng = np.random.default_rng(3)
    n, N = 5, 3
    Vi = rng.integers(-4, 5, size=(n, N))
    Di = rng.integers(-6, 7, size=(n, N))
    ri = rng.integers(1, 5, size=n)
    # V = Vi / 4, r = ri / 2: exactly representable in binary FP64.
    V = [[Fraction(int(Vi[i, j]), 4) for j in range(N)] for i in range(n)]
    W = [[(Fraction(int(ri[i]), 2) if i == j else Fraction(0)) + sum(V[i][l] * V[j][l] for l in range(N))
          for j in range(n)] for i in range(n)]
    Zx = _exact_solve(W, [[int(Di[i, k]) for k in range(N)] for i in range(n)])
    Zx = np.array([[float(v) for v in row] for row in Zx])
    out = oracle.sm_solve(ri / 2.0, Vi / 4.0, Di.astype(float))
    assert _rel(out["Z"], Zx) < 1e-14


# --- the paper's recursive definition S(x, k) (Section 3, eq. recursive-SMF) -
def _S(x, k, r, V):
    if k == 0:
        return x / r
    v = V[:, k - 1]
    f = _S(x, k - 1, r, V)
    g = _S(v, k - 1, r, V)
    return f - g * (v @ f) / (1.0 + v @ g)


@pytest.mark.parametrize("n,N", [(6, 1), (9, 4), (12, 7)])
def test_matches_recursive_definition(n, N):
    r, V, D = _problem(n, N, seed=11 + N)
    Zrec = np.column_stack([_S(D[:, j], N, r, V) for j in range(N)])
    out = oracle.sm_solve(r, V, D)
    assert _rel(out["Z"], Zrec) < 1e-13


def test_rank_one_closed_form():
    # N = 1: one application of the Sherman-Morrison identity to R + v v^T.
    n = 25
    r, V, D = _problem(n, 1, seed=5, nrhs=4)
    v = V[:, 0]
    Rinv_D = D / r[:, None]
    Rinv_v = v / r
    Zcf = Rinv_D - np.outer(Rinv_v, v @ Rinv_D) / (1.0 + v @ Rinv_v)
    out = oracle.sm_solve(r, V, D)
    assert _rel(out["Z"], Zcf) < 1e-14


# --- W^{-1} is symmetric (the SM product form is not manifestly so) --------
def test_inverse_is_symmetric():
    n, N = 48, 12
    r, V, _ = _problem(n, N, seed=21)
    out = oracle.sm_solve(r, V, np.eye(n))
    A = out["Z"]
    assert np.linalg.norm(A - A.T) / np.linalg.norm(A) < 1e-14
    W = np.diag(r) + V @ V.T
    assert np.linalg.norm(A @ W - np.eye(n)) < 1e-12


# --- pivots: Theorem 2, the determinant lemma, the LDL^T pivots of C --------
def test_gamma_properties():
    n, N = 80, 16
    r, V, D = _problem(n, N, seed=31)
    g = oracle.sm_solve(r, V, D)["gamma"]
    assert np.all(g > 1.0)
    C = np.eye(N) + V.T @ (V / r[:, None])
    sign, logdet = np.linalg.slogdet(C)
    assert sign > 0 and abs(np.sum(np.log(g)) - logdet) < 1e-12 * max(1.0, abs(logdet))
    L = np.linalg.cholesky(C)
    assert np.allclose(g, np.diag(L) ** 2, rtol=1e-13, atol=0)


def test_zero_anomaly_column_is_noop():
    n, N = 30, 6
    r, V, D = _problem(n, N, seed=41)
    V0 = V.copy()
    V0[:, 2] = 0.0
    out = oracle.sm_solve(r, V0, D)
    assert out["gamma"][2] == 1.0
    ref = oracle.sm_solve(r, np.delete(V0, 2, axis=1), D)
    assert _rel(out["Z"], ref["Z"]) < 1e-14


def test_duplicate_columns():
    n, N = 40, 5
    r, V, D = _problem(n, N, seed=43)
    V[:, 3] = V[:, 1]
    out = oracle.sm_solve(r, V, D)
    assert _rel(out["Z"], _dense_solve(r, V, D)) < 1e-12


def test_column_order_invariance():
    n, N = 70, 11
    r, V, D = _problem(n, N, seed=51)
    p = np.random.default_rng(0).permutation(N)
    a = oracle.sm_solve(r, V, D)["Z"]
    b = oracle.sm_solve(r, V[:, p], D)["Z"]
    assert _rel(a, b) < 1e-13


# --- operation counts of Section 3.2 and Section 3.4 -------------------------
@pytest.mark.parametrize("n,N", [(10, 1), (37, 9), (16, 40)])
def test_long_operation_counts(n, N):
    r, V, D = _problem(n, N, seed=61)
    assert oracle.sm_solve(r, V, D)["longops"] == 3 * (N * N * n + N * n)
    # pivoting: 3(N^2 n + N n) + sum_k k n = 3.5 (N^2 n + N n)
    assert 2 * oracle.sm_solve(r, V, D, pivot=True)["longops"] == 7 * (N * N * n + N * n)


# --- pivoting (Section 3.4) ---------------------------------------------------
def test_pivoting_same_solution_and_greedy_pivots():
    n, N = 90, 14
    r, V, D = _problem(n, N, seed=71, v_scale=3.0)
    a = oracle.sm_solve(r, V, D)
    b = oracle.sm_solve(r, V, D, pivot=True)
    assert _rel(b["Z"], a["Z"]) < 1e-12
    perm = b["perm"]
    assert sorted(perm.tolist()) == list(range(N))
    first = 1.0 + np.sum(V * (V / r[:, None]), axis=0)
    assert perm[0] == int(np.argmax(first))
    assert abs(b["gamma"][0] - first.max()) < 1e-12 * first.max()
    # every candidate value only decreases as W^{(k)} grows, so the greedy
    # sequence of pivots is non-increasing.
    assert np.all(np.diff(b["gamma"]) <= 1e-12 * b["gamma"][:-1])
    # the product of pivots is order independent (determinant lemma).
    assert abs(np.sum(np.log(a["gamma"])) - np.sum(np.log(b["gamma"]))) < 1e-12


# --- apply-only with a stored factor ------------------------------------------
def test_apply_matches_solve():
    n, N = 64, 10
    r, V, D = _problem(n, N, seed=81)
    f = oracle.sm_solve(r, V, D, want_factor=True)
    D2 = synth.normal(9, 3, n * 4).reshape(4, n).T
    Y = oracle.sm_apply(r, V, f["U"], f["gamma"], D2)
    assert _rel(Y, _dense_solve(r, V, D2)) < 1e-12
    fp = oracle.sm_solve(r, V * np.linspace(0.2, 3.0, N), D, pivot=True, want_factor=True)
    Yp = oracle.sm_apply(r, V * np.linspace(0.2, 3.0, N), fp["U"], fp["gamma"], D2, perm=fp["perm"])
    assert _rel(Yp, _dense_solve(r, V * np.linspace(0.2, 3.0, N), D2)) < 1e-12


def test_residual_definition():
    n, N = 33, 7
    r, V, D = _problem(n, N, seed=91)
    Z = synth.normal(1, 2, n * N).reshape(N, n).T
    W = np.diag(r) + V @ V.T
    assert _rel(oracle.residual(r, V, Z, D), D - W @ Z) < 1e-13


# --- failure modes of Section 3.3 ---------------------------------------------
def test_rejects_nonpositive_r():
    r, V, D = _problem(10, 3, seed=1)
    for bad in (0.0, -1.0, np.nan, np.inf):
        rr = r.copy()
        rr[4] = bad
        with pytest.raises(oracle.OracleError) as e:
            oracle.sm_solve(rr, V, D)
        assert e.value.code == 2


def test_rejects_nonfinite_v():
    r, V, D = _problem(10, 3, seed=1)
    V[2, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.sm_solve(r, V, D)
    assert e.value.code == 2


# --- building V and D from the ensemble, and the analysis update --------------
def _tiny_ensemble(n_state=14, N=6, seed=5):
    truth, XB = synth.lorenz_ensemble(n_state, N, seed, spinup=200, steps=5)
    obs_idx = np.array([0, 3, 4, 9, 13], dtype=np.int64)
    n = obs_idx.size
    r = synth.uniform(seed, synth.P_RDIAG, n, 0.005, 0.02)
    y = truth[obs_idx] + np.sqrt(r) * synth.normal(seed, synth.P_OBS, n)
    E = np.asfortranarray(synth.normal(seed, synth.P_EPERT, n * N).reshape(N, n).T * np.sqrt(r)[:, None])
    H = np.zeros((n, n_state))
    H[np.arange(n), obs_idx] = 1.0
    return truth, XB, obs_idx, r, y, E, H


def test_build_vd_against_sample_covariance():
    truth, XB, obs_idx, r, y, E, H = _tiny_ensemble()
    V, D = oracle.build_vd(XB, obs_idx, y, E)
    P = np.cov(XB, ddof=1)          # sample covariance, Section 2
    assert _rel(V @ V.T, H @ P @ H.T) < 1e-13
    assert np.abs(V.sum(axis=1)).max() < 1e-14 * np.abs(V).max() * V.shape[1]
    Y = y[:, None] + E
    assert _rel(D, Y - H @ XB) < 1e-15


def test_analysis_against_kalman_gain_form():
    truth, XB, obs_idx, r, y, E, H = _tiny_ensemble()
    V, D = oracle.build_vd(XB, obs_idx, y, E)
    Z = oracle.sm_solve(r, V, D)["Z"]
    XA = oracle.analysis(XB, V, Z)
    P = np.cov(XB, ddof=1)
    K = P @ H.T @ np.linalg.inv(H @ P @ H.T + np.diag(r))   # eq. EnKF:kalman-gain
    XA_ref = XB + K @ (y[:, None] + E - H @ XB)              # eq. EnKF:ensemble-analysis
    assert _rel(XA - XB, XA_ref - XB) < 1e-11


def test_local_analysis_against_dense():
    n_glob, N, P = 48, 8, 20
    truth, XB = synth.lorenz_ensemble(n_glob, N, 17, spinup=100, steps=3)
    r = np.full(n_glob, 0.01)
    y = truth + 0.1 * synth.normal(17, synth.P_OBS, n_glob)
    E = np.asfortranarray(0.1 * synth.normal(17, synth.P_EPERT, n_glob * N).reshape(N, n_glob).T)
    V, D = oracle.build_vd(XB, np.arange(n_glob), y, E)
    start, ln, pts = synth.local_windows(n_glob, P, 17, lo=1, hi=n_glob)
    xa = oracle.local_analysis(r, V, D, XB, start, ln, pts)
    for p in range(P):
        rows = (start[p] + np.arange(ln[p])) % n_glob
        Zp = _dense_solve(r[rows], V[rows], D[rows])
        s = pts[p]
        dx = (XB[s] - XB[s].mean()) / np.sqrt(N - 1)
        ref = XB[s] + dx @ (V[rows].T @ Zp)
        assert np.allclose(xa[p], ref, rtol=1e-12, atol=1e-13)


def test_analysis_reduces_error_when_spread_matches_error():
    # A statistically consistent background: mean error and member spread are
    # both N(0, sb^2); observations carry N(0, so^2). The analysis mean must
    # then be closer to the truth than the background mean (Section 2).
    n_state, N, sb, so = 30, 400, 0.5, 0.1
    truth = synth.uniform(3, synth.P_TRUTH0, n_state, -5, 5)
    xb = truth + sb * synth.normal(3, synth.P_XPERT, n_state)
    XB = np.asfortranarray(xb[:, None] + sb * synth.normal(3, synth.P_MEMBER, n_state * N).reshape(N, n_state).T)
    obs = np.arange(0, n_state, 2, dtype=np.int64)
    n = obs.size
    r = np.full(n, so * so)
    y = truth[obs] + so * synth.normal(3, synth.P_OBS, n)
    E = np.asfortranarray(so * synth.normal(3, synth.P_EPERT, n * N).reshape(N, n).T)
    V, D = oracle.build_vd(XB, obs, y, E)
    XA = oracle.analysis(XB, V, oracle.sm_solve(r, V, D)["Z"])
    rmse_b = np.sqrt(np.mean((XB.mean(axis=1) - truth)[obs] ** 2))
    rmse_a = np.sqrt(np.mean((XA.mean(axis=1) - truth)[obs] ** 2))
    assert rmse_a < 0.5 * rmse_b


# --- the pins catch plausible mistakes planted in a copy of the oracle -------
MUTANTS = [
    ("zj[i] -= h[i] * c;", "zj[i] += h[i] * c;"),                                  # wrong sign
    ("double g = 1.0 + dot_col(n, vk, uk);", "double g = dot_col(n, vk, uk);"),    # dropped term
    ("AT(U, n, i, j) = AT(Vw, n, i, j) / r[i];", "AT(U, n, i, j) = AT(Vw, n, i, j) * r[i];"),
    ("for (int32_t j = k + 1; j < N; ++j) {", "for (int32_t j = k + 2; j < N; ++j) {"),  # index
    ("for (int64_t i = 0; i < n; ++i) h[i] = uk[i] / g;", "for (int64_t i = 0; i < n; ++i) h[i] = uk[i];"),
    ("double c = dot_col(n, vk, zj);", "double c = dot_col(n, &AT(U, n, 0, k), zj);"),  # swapped operand
]


@pytest.mark.parametrize("before,after", MUTANTS)
def test_pins_catch_planted_mistakes(tmp_path, before, after):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "enkf_oracle.c")).read()
    assert src.count(before) == 1
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    (mdir / "enkf_oracle.c").write_text(src.replace(before, after))
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "__init__.py"), mdir / "__init__.py")
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(1, %r)\n"
        "import numpy as np, scipy.linalg as sla, oracle, synth\n"
        "r, V, D = synth.small_vd(40, 9, 3)\n"
        "W = np.diag(r) + V @ V.T\n"
        "Z = oracle.sm_solve(r, V, D)['Z']\n"
        "ref = sla.solve(W, D, assume_a='pos')\n"
        "print(np.linalg.norm(Z - ref) / np.linalg.norm(ref))\n"
    ) % (str(tmp_path), os.path.dirname(os.path.dirname(oracle.__file__)))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert float(res.stdout.strip().splitlines()[-1]) > 1e-6
