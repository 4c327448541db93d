"""FP64 CPU oracle for the EnKF analysis by the iterative Sherman-Morrison formula.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The GPU library never imports, links or
calls anything here, and this package imports nothing from it.

The arithmetic lives in ``enkf_oracle.c`` (plain C, FP64, no BLAS, built with
-ffp-contract=off); this module compiles it with gcc and marshals numpy arrays.
Each function cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "enkf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS = {0: "ok", 1: "invalid argument", 2: "not positive definite", 3: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}")
        self.code = code


def build() -> str:
    """Compile the oracle (gcc -O2 -fopenmp -ffp-contract=off)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", _SRC, "-o", _LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_sm_solve.argtypes = [i64, i32, vp, vp, i64, vp, i64, i32, vp, i64, vp, vp, i32, vp, vp]
    lib.oracle_sm_apply.argtypes = [i64, i32, vp, vp, i64, vp, vp, vp, vp, i64, i32, vp, i64]
    lib.oracle_residual.argtypes = [i64, i32, vp, vp, i64, vp, i64, vp, i64, i32, vp, i64]
    lib.oracle_build_vd.argtypes = [i64, i32, vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, i64]
    lib.oracle_analysis.argtypes = [i64, i32, i64, vp, i64, vp, i64, vp, i64, vp, i64]
    lib.oracle_local_analysis.argtypes = [i64, i32, vp, vp, i64, vp, i64, i64, vp, i64, i64, vp, vp, vp, vp, i64]
    lib.oracle_localized_analysis.argtypes = [i64, i32, i64, vp, i64, vp, i64, vp, i64, vp, ctypes.c_double, i64,
                                              i64, vp, i64]
    lib.oracle_sm_solve_block_r.argtypes = [i64, i32, i64, vp, vp, vp, i64, vp, i64, i32, vp, i64, vp]
    lib.oracle_l96_rk4.argtypes = [i64, i64, vp, i64, i64, ctypes.c_double, ctypes.c_double]
    lib.oracle_localized_rows.argtypes = [i64, i32, i64, vp, i64, vp, i64, vp, i64, vp, ctypes.c_double, i64, i64,
                                          i64, i64, vp, i64]
    for f in ("oracle_sm_solve", "oracle_sm_apply", "oracle_residual", "oracle_build_vd",
              "oracle_analysis", "oracle_local_analysis", "oracle_localized_analysis", "oracle_localized_rows",
              "oracle_sm_solve_block_r", "oracle_l96_rk4"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a, shape_dims=2) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1 and shape_dims == 2:
        a = a[:, None]
    return np.asfortranarray(a)


def _check(code: int, where: str):
    if code != 0:
        raise OracleError(code, where)


def sm_solve(r, V, D, pivot: bool = False, want_factor: bool = False):
    """Iterative Sherman-Morrison solve S*(R, V, D) (Section 3.1, Steps 1-2;
    pivoting of Section 3.4 when ``pivot``).

    Returns a dict with Z, gamma, perm, longops and, when ``want_factor``,
    U (column k = u_k^{(k-1)})."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    V = _f64(V)
    D = _f64(D)
    n, N = V.shape
    nrhs = D.shape[1]
    assert r.shape == (n,) and D.shape[0] == n
    Z = np.zeros((n, nrhs), dtype=np.float64, order="F")
    U = np.zeros((n, N), dtype=np.float64, order="F") if want_factor else None
    gamma = np.zeros(N, dtype=np.float64)
    perm = np.zeros(N, dtype=np.int32)
    ops = ctypes.c_int64(0)
    code = _load().oracle_sm_solve(n, N, _p(r), _p(V), n, _p(D), n, nrhs, _p(Z), n, _p(U), _p(gamma),
                                   1 if pivot else 0, _p(perm), ctypes.byref(ops))
    _check(code, "oracle_sm_solve")
    return {"Z": Z, "gamma": gamma, "perm": perm, "longops": int(ops.value), "U": U}


def pack_blocks(blocks):
    """Offsets (nblk + 1) and the column-major blocks packed one after the
    other, the layout of a block-diagonal R used by the solvers."""
    sizes = [b.shape[0] for b in blocks]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    packed = np.concatenate([np.asarray(b, dtype=np.float64).ravel(order="F") for b in blocks])
    return off, packed


def sm_solve_block_r(blocks, V, D):
    """Iterative Sherman-Morrison solve with a block-diagonal R = diag(blocks)
    (Section 2.1; Step 1 block by block, Section 3.1). Returns Z and gamma."""
    off, packed = pack_blocks(blocks)
    V, D = _f64(V), _f64(D)
    n, N = V.shape
    nrhs = D.shape[1]
    assert off[-1] == n
    Z = np.zeros((n, nrhs), dtype=np.float64, order="F")
    gamma = np.zeros(N, dtype=np.float64)
    code = _load().oracle_sm_solve_block_r(n, N, len(blocks), _p(off), _p(packed), _p(V), n, _p(D), n, nrhs,
                                           _p(Z), n, _p(gamma))
    _check(code, "oracle_sm_solve_block_r")
    return {"Z": Z, "gamma": gamma}


def sm_apply(r, V, U, gamma, X, perm=None):
    """Z-half of S*: Step 1 and the Z-update of every level with a stored
    factor (Section 3.1, eq. SM-step-2-Z)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    V, U, X = _f64(V), _f64(U), _f64(X)
    n, N = V.shape
    Y = np.zeros_like(X, order="F")
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    code = _load().oracle_sm_apply(n, N, _p(r), _p(V), n, _p(U), _p(g), _p(pm), _p(X), n, X.shape[1], _p(Y), n)
    _check(code, "oracle_sm_apply")
    return Y


def residual(r, V, Z, D):
    """rho = D - (R Z + V (V^T Z)) for the system of eq. EnKSM:system-to-solve-V."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    V, Z, D = _f64(V), _f64(Z), _f64(D)
    n, N = V.shape
    rho = np.zeros_like(D, order="F")
    code = _load().oracle_residual(n, N, _p(r), _p(V), n, _p(Z), n, _p(D), n, D.shape[1], _p(rho), n)
    _check(code, "oracle_residual")
    return rho


def build_vd(XB, obs_idx, y, E):
    """V = H S and D = Y - H X^B (Section 3, eq. EnKSM:system-rewritten)."""
    XB, E = _f64(XB), _f64(E)
    obs = np.ascontiguousarray(obs_idx, dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n_state, N = XB.shape
    n = obs.shape[0]
    V = np.zeros((n, N), order="F")
    D = np.zeros((n, N), order="F")
    code = _load().oracle_build_vd(n_state, N, _p(XB), n_state, _p(obs), n, _p(y), _p(E), n, _p(V), n, _p(D), n)
    _check(code, "oracle_build_vd")
    return V, D


def analysis(XB, V, Z):
    """X^A = X^B + S V^T Z (Section 3.1)."""
    XB, V, Z = _f64(XB), _f64(V), _f64(Z)
    n_state, N = XB.shape
    n = V.shape[0]
    XA = np.zeros_like(XB, order="F")
    code = _load().oracle_analysis(n_state, N, n, _p(XB), n_state, _p(V), n, _p(Z), n, _p(XA), n_state)
    _check(code, "oracle_analysis")
    return XA


def localized_analysis(XB, V, Z, loc, length, radius=-1, ring=0):
    """Partial localization (Section 3.1.2, eq. localized-correction-component):
    X^A = X^B + (Delta o (S V^T)) Z with delta(i, j) = exp(-d(i, loc_j)/length),
    zero past `radius` (radius < 0: none), d taken on a ring of `ring` points
    (ring = 0: no wrap)."""
    XB, V, Z = _f64(XB), _f64(V), _f64(Z)
    lc = np.ascontiguousarray(loc, dtype=np.int64)
    n_state, N = XB.shape
    n = V.shape[0]
    XA = np.zeros_like(XB, order="F")
    code = _load().oracle_localized_analysis(n_state, N, n, _p(XB), n_state, _p(V), n, _p(Z), n, _p(lc),
                                             ctypes.c_double(float(length)), int(radius), int(ring), _p(XA), n_state)
    _check(code, "oracle_localized_analysis")
    return XA


def localized_rows(XB, V, Z, loc, length, radius, ring, row_begin, row_end):
    """Rows [row_begin, row_end) of localized_analysis (the rows are
    independent); returns those rows only."""
    XB, V, Z = _f64(XB), _f64(V), _f64(Z)
    lc = np.ascontiguousarray(loc, dtype=np.int64)
    n_state, N = XB.shape
    n = V.shape[0]
    XA = np.zeros_like(XB, order="F")
    code = _load().oracle_localized_rows(n_state, N, n, _p(XB), n_state, _p(V), n, _p(Z), n, _p(lc),
                                         ctypes.c_double(float(length)), int(radius), int(ring), int(row_begin),
                                         int(row_end), _p(XA), n_state)
    _check(code, "oracle_localized_rows")
    return XA[row_begin:row_end]


def l96_forecast(X, nsteps, F=8.0, dt=0.05):
    """Lorenz-96 RK4 forecast of every column of X (a copy is returned)."""
    X = np.array(X, dtype=np.float64, order="F", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    n, m = X.shape
    _check(_load().oracle_l96_rk4(n, m, _p(X), n, int(nsteps), float(F), float(dt)), "oracle_l96_rk4")
    return X


def cycle_l96(XB0, obs_idx, ys, Es, r, nsteps, F=8.0, dt=0.05, localize=None, truths=None):
    """The cycling filter of the Lorenz-96 experiments (Section 4): per cycle
    c, forecast the ensemble nsteps RK4 steps, build V and D from the
    perturbed observations ys[c] + Es[c] (Section 2), solve with the
    iterative Sherman-Morrison formula (Section 3.1) and update the ensemble,
    with the partial localization of Section 3.1.2 when
    localize = (length, ring). Returns the final ensemble and, with truths,
    the forecast and analysis RMSE of the ensemble mean per cycle."""
    XB = np.array(XB0, dtype=np.float64, order="F", copy=True)
    rmse_f, rmse_a = [], []
    for c in range(len(ys)):
        XB = l96_forecast(XB, nsteps, F, dt)
        V, D = build_vd(XB, obs_idx, ys[c], Es[c])
        Z = sm_solve(r, V, D)["Z"]
        if localize is None:
            XA = analysis(XB, V, Z)
        else:
            XA = localized_analysis(XB, V, Z, obs_idx, localize[0], -1, localize[1])
        if truths is not None:
            rmse_f.append(float(np.sqrt(np.mean((XB.mean(axis=1) - truths[c]) ** 2))))
            rmse_a.append(float(np.sqrt(np.mean((XA.mean(axis=1) - truths[c]) ** 2))))
        XB = XA
    return XB, rmse_f, rmse_a


def local_analysis(r, V, D, XB, win_start, win_len, state_idx):
    """Independent localized analyses over cyclic observation windows; returns
    the analysed state points (n_prob x N)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    V, D, XB = _f64(V), _f64(D), _f64(XB)
    ws = np.ascontiguousarray(win_start, dtype=np.int64)
    wl = np.ascontiguousarray(win_len, dtype=np.int64)
    si = np.ascontiguousarray(state_idx, dtype=np.int64)
    n_glob, N = V.shape
    n_state = XB.shape[0]
    P = ws.shape[0]
    xa = np.zeros((P, N), order="F")
    code = _load().oracle_local_analysis(n_glob, N, _p(r), _p(V), n_glob, _p(D), n_glob, n_state, _p(XB),
                                         n_state, P, _p(ws), _p(wl), _p(si), _p(xa), max(P, 1))
    _check(code, "oracle_local_analysis")
    return xa


# ---------------------------------------------------------------------------
# Diagnostics used by the parity gates (plain numpy on top of the C results).
# ---------------------------------------------------------------------------
def rel_residual(r, V, Z, D) -> float:
    """||D - W Z||_F / ||D||_F."""
    rho = residual(r, V, Z, D)
    return float(np.linalg.norm(rho) / np.linalg.norm(D))


def norm_w_estimate(r, V) -> float:
    """Upper estimate of ||W||_2 = ||R + V V^T||_2: max r + sigma_max(V)^2,
    sigma_max^2 the largest eigenvalue of the N x N Gram V^T V."""
    V = np.asarray(V, dtype=np.float64)
    gram = V.T @ V
    return float(np.max(r) + np.max(np.linalg.eigvalsh(0.5 * (gram + gram.T))))


def backward_error(r, V, Z, D) -> float:
    """eta = ||D - W Z||_F / (||W||_2 ||Z||_F + ||D||_F)."""
    rho = residual(r, V, Z, D)
    return float(np.linalg.norm(rho) / (norm_w_estimate(r, V) * np.linalg.norm(Z) + np.linalg.norm(D)))
