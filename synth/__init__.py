"""Seeded synthetic inputs for the EnKF analysis workloads.

Holds no arithmetic of the analysis method: only random streams
(Philox4x64-10 + Box-Muller, in ``synth.c``), the Lorenz-96 model advanced by
RK4, and the recipes that shape the five workloads. Both the HIP path and the
FP64 oracle take their inputs from here; neither is imported by this module.

All matrices are column-major (numpy order ``"F"``), one column per ensemble
member, as in the paper's definition of the background ensemble (Section 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# Stream purposes: each random quantity draws from its own keyed stream.
P_TRUTH0, P_MEMBER, P_OBS, P_EPERT, P_RDIAG, P_VDRAW, P_VROW, P_DDRAW, P_NP, P_XPERT = range(1, 11)
SEED_BASE = 20130212


def build() -> str:
    """Compile synth.c into libsynth.so (gcc, OpenMP, no FP contraction)."""
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
    u64, i64, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    vp = ctypes.c_void_p
    lib.synth_philox4x64.argtypes = [vp, vp, vp]
    lib.synth_uniform.argtypes = [u64, u64, i64, i64, dbl, dbl, vp]
    lib.synth_normal.argtypes = [u64, u64, i64, i64, vp]
    lib.synth_randint.argtypes = [u64, u64, i64, i64, i64, i64, vp]
    lib.synth_l96_advance.argtypes = [i64, vp, dbl, dbl, i64]
    lib.synth_l96_advance.restype = ctypes.c_int
    lib.synth_l96_advance_members.argtypes = [i64, i64, vp, i64, dbl, dbl, i64]
    lib.synth_l96_advance_members.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().synth_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, purpose: int, count: int, lo=0.0, hi=1.0, offset: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().synth_uniform(seed, purpose, offset, count, lo, hi, _ptr(out))
    return out


def normal(seed: int, purpose: int, count: int, offset: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().synth_normal(seed, purpose, offset, count, _ptr(out))
    return out


def randint(seed: int, purpose: int, count: int, lo: int, hi: int, offset: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    _load().synth_randint(seed, purpose, offset, count, lo, hi, _ptr(out))
    return out


def l96_advance(x: np.ndarray, nsteps: int, F: float = 8.0, dt: float = 0.05) -> np.ndarray:
    """Advance one Lorenz-96 state in place by nsteps RK4 steps."""
    assert x.dtype == np.float64 and x.flags.c_contiguous and x.ndim == 1
    if _load().synth_l96_advance(x.shape[0], _ptr(x), F, dt, nsteps) != 0:
        raise MemoryError("synth_l96_advance: no scratch")
    return x


def l96_advance_members(X: np.ndarray, nsteps: int, F: float = 8.0, dt: float = 0.05) -> np.ndarray:
    """Advance every column of X (F-order) in place."""
    assert X.dtype == np.float64 and X.flags.f_contiguous and X.ndim == 2
    n, m = X.shape
    if _load().synth_l96_advance_members(n, m, _ptr(X), n, F, dt, nsteps) != 0:
        raise MemoryError("synth_l96_advance_members: no scratch")
    return X


@dataclass
class Workload:
    """One synthetic analysis problem. Arrays are float64, column-major."""
    name: str
    n_state: int
    n_ens: int
    n_obs: int
    seed: int
    r: np.ndarray                       # (n_obs,) diagonal of R, > 0
    XB: Optional[np.ndarray] = None     # (n_state, N) background ensemble
    obs_idx: Optional[np.ndarray] = None  # (n_obs,) int64 rows of XB observed by H
    y: Optional[np.ndarray] = None      # (n_obs,) observations
    E: Optional[np.ndarray] = None      # (n_obs, N) observation perturbations ~ N(0, R)
    truth: Optional[np.ndarray] = None  # (n_state,)
    V: Optional[np.ndarray] = None      # (n_obs, N) given directly (no XB)
    D: Optional[np.ndarray] = None      # (n_obs, N) given directly (no XB)
    extra: dict = field(default_factory=dict)


def lorenz_ensemble(n_state: int, n_ens: int, seed: int, spinup: int = 1000, steps: int = 10,
                    sigma: float = 0.05, F: float = 8.0, dt: float = 0.05):
    """Truth from U(-1,1) spun up `spinup` RK4 steps; members = truth +
    N(0, sigma^2) per component; then members and truth advance `steps`."""
    truth = uniform(seed, P_TRUTH0, n_state, -1.0, 1.0)
    l96_advance(truth, spinup, F, dt)
    pert = normal(seed, P_MEMBER, n_state * n_ens).reshape(n_ens, n_state).T
    XB = np.asfortranarray(truth[:, None] + sigma * pert)
    del pert
    l96_advance_members(XB, steps, F, dt)
    l96_advance(truth, steps, F, dt)
    return truth, XB


def lorenz_workload(name: str, n_state: int, n_ens: int, obs_stride: int, seed: int,
                    r_const: Optional[float] = None, r_range=(0.005, 0.02),
                    spinup: int = 1000, steps: int = 10) -> Workload:
    """Lorenz-96 ring workload: H selects every `obs_stride`-th variable
    (rows 0, s, 2s, ...); R diagonal, constant or U(r_range); y = H truth +
    N(0, R); perturbed observations E ~ N(0, R) independently per member."""
    truth, XB = lorenz_ensemble(n_state, n_ens, seed, spinup, steps)
    obs_idx = np.arange(0, n_state, obs_stride, dtype=np.int64)
    n_obs = obs_idx.shape[0]
    if r_const is not None:
        r = np.full(n_obs, float(r_const))
    else:
        r = uniform(seed, P_RDIAG, n_obs, r_range[0], r_range[1])
    sd = np.sqrt(r)
    y = truth[obs_idx] + sd * normal(seed, P_OBS, n_obs)
    E = normal(seed, P_EPERT, n_obs * n_ens).reshape(n_ens, n_obs).T * sd[:, None]
    E = np.asfortranarray(E)
    return Workload(name, n_state, n_ens, n_obs, seed, r, XB=XB, obs_idx=obs_idx, y=y, E=E, truth=truth)


def direct_vd_workload(name: str, n_obs: int, n_ens: int, seed: int, row_scale=(0.5, 2.0),
                       r_range=(0.01, 0.1)) -> Workload:
    """V and D drawn directly: V_ij = g_ij s_i / sqrt(N-1) with g ~ N(0,1) and
    per-row s_i ~ U(row_scale); R = diag(U(r_range)); D_ij ~ N(0,1)."""
    s = uniform(seed, P_VROW, n_obs, row_scale[0], row_scale[1])
    g = normal(seed, P_VDRAW, n_obs * n_ens).reshape(n_ens, n_obs).T
    V = np.asfortranarray(g * (s / np.sqrt(max(n_ens - 1, 1)))[:, None])
    del g
    D = np.asfortranarray(normal(seed, P_DDRAW, n_obs * n_ens).reshape(n_ens, n_obs).T)
    r = uniform(seed, P_RDIAG, n_obs, r_range[0], r_range[1])
    return Workload(name, 0, n_ens, n_obs, seed, r, V=V, D=D)


def local_windows(n_glob: int, n_prob: int, seed: int, lo: int = 16, hi: int = 512):
    """Localized problem p observes the n_p consecutive ring points starting at
    (p - n_p // 2) mod n_glob, with n_p ~ U{lo..hi}; its state point is p."""
    n_p = randint(seed, P_NP, n_prob, lo, hi)
    p = np.arange(n_prob, dtype=np.int64)
    start = np.mod(p - n_p // 2, n_glob).astype(np.int64)
    return start, n_p.astype(np.int64), p


# ---------------------------------------------------------------------------
# The five workloads. Sizes follow the workload table; the seed of workload c
# is SEED_BASE + c.
# ---------------------------------------------------------------------------
def c1(seed: Optional[int] = None) -> Workload:
    """n_state=40, N=20, every other variable observed, R = 0.01 I."""
    return lorenz_workload("c1", 40, 20, 2, SEED_BASE + 1 if seed is None else seed, r_const=0.01)


def c2(seed: Optional[int] = None, n_state: int = 1_048_576, n_ens: int = 96) -> Workload:
    """n_state=1,048,576, N=96, every 4th variable observed, r ~ U(0.005,0.02)."""
    return lorenz_workload("c2", n_state, n_ens, 4, SEED_BASE + 2 if seed is None else seed)


def c3(seed: Optional[int] = None, n_obs: int = 2_097_152, n_ens: int = 256) -> Workload:
    """n_obs=2,097,152, N=256, V and D drawn directly."""
    return direct_vd_workload("c3", n_obs, n_ens, SEED_BASE + 3 if seed is None else seed)


def c4(seed: Optional[int] = None, n_state: int = 4096, n_ens: int = 64, n_prob: int = 4096,
       lo: int = 16, hi: int = 512) -> Workload:
    """Ring n_state=4096, N=64, H = I, R = 0.01 I; n_prob local problems."""
    s = SEED_BASE + 4 if seed is None else seed
    w = lorenz_workload("c4", n_state, n_ens, 1, s, r_const=0.01)
    start, n_p, pts = local_windows(n_state, n_prob, s, lo, hi)
    w.extra.update(win_start=start, win_len=n_p, state_idx=pts)
    return w


def c5(seed: Optional[int] = None, n_state: int = 2_097_152, n_ens: int = 1024) -> Workload:
    """n_state=2,097,152, N=1024, every 4th variable observed, r ~ U(0.005,0.02)."""
    return lorenz_workload("c5", n_state, n_ens, 4, SEED_BASE + 5 if seed is None else seed)


def c6(seed: Optional[int] = None, n_state: int = 32_768, n_ens: int = 64) -> Workload:
    """Partial localization workload: Lorenz-96 ring n_state=32,768, N=64,
    every 2nd variable observed (n_obs=16,384), r ~ U(0.005,0.02)."""
    return lorenz_workload("c6", n_state, n_ens, 2, SEED_BASE + 6 if seed is None else seed)


def l96_cycle_inputs(n_state: int, n_ens: int, cycles: int, nsteps: int, seed: int, sd_obs: float = 0.01,
                     bg_err: float = 0.05):
    """Inputs of a Lorenz-96 cycling run in the setting of the paper's
    Lorenz-96 experiments: H = I (n_obs = n_state), R = sd_obs^2 I, truth spun
    up 1000 steps from a seeded start, members = truth (1 + bg_err g) with g
    ~ N(0, 1) (a 5% background error), then per cycle the truth advanced
    nsteps RK4 steps, y = truth + N(0, R) and perturbations E ~ N(0, R).
    Returns (XB0, obs_idx, r, truths, ys, Es)."""
    truth = l96_advance(np.ascontiguousarray(8.0 + normal(seed, P_TRUTH0, n_state)), 1000)
    g = normal(seed, P_MEMBER, n_state * n_ens).reshape(n_ens, n_state).T
    XB = np.asfortranarray(truth[:, None] * (1.0 + bg_err * g))
    obs = np.arange(n_state, dtype=np.int64)
    r = np.full(n_state, sd_obs ** 2)
    truths, ys, Es = [], [], []
    t = truth.copy()
    for c in range(cycles):
        t = l96_advance(t, nsteps)
        truths.append(t.copy())
        ys.append(t + sd_obs * normal(seed, P_OBS, n_state, offset=c * n_state))
        e = normal(seed, P_EPERT, n_state * n_ens, offset=c * n_state * n_ens)
        Es.append(np.asfortranarray(sd_obs * e.reshape(n_ens, n_state).T))
    return XB, obs, r, truths, ys, Es


def small_vd(n_obs: int, n_ens: int, seed: int, r_range=(0.5, 2.0), v_scale: float = 1.0,
             nrhs: Optional[int] = None):
    """Small random (r, V, D) for checks: V ~ v_scale N(0,1)/sqrt(N), D ~ N(0,1)."""
    nrhs = n_ens if nrhs is None else nrhs
    V = np.asfortranarray(normal(seed, P_VDRAW, n_obs * n_ens).reshape(n_ens, n_obs).T
                          * (v_scale / np.sqrt(max(n_ens, 1))))
    D = np.asfortranarray(normal(seed, P_DDRAW, n_obs * nrhs).reshape(nrhs, n_obs).T)
    r = uniform(seed, P_RDIAG, n_obs, r_range[0], r_range[1])
    return r, V, D
