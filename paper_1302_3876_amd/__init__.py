"""Python binding of the MI355X EnKF analysis library (``libenkf_sm.so``).

Argument marshalling only: every step of the analysis runs in the library's
HIP kernels. Functions keep the names of the C ABI in ``include/enkf_sm.h``
and take torch CUDA tensors (PyTorch provides device memory and the stream:
calls are enqueued on ``torch.cuda.current_stream()``). Matrices are
column-major: a 2-D tensor of shape (rows, cols) with ``stride(0) == 1``;
``colmajor`` allocates one.

If the shared library is not built this module raises on first use; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libenkf_sm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "enkf_sm.h")
HEADER_LOCAL = os.path.join(os.path.dirname(HERE), "include", "enkf_local.h")

ENKF_F64, ENKF_F32 = 0, 1
ENKF_SM_PLAIN, ENKF_SM_BLOCKED = 0, 1
MATH = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16x3": 4, "f16x2": 5}
ENKF_FLAG_PIVOT = 0x1
ENKF_FLAG_DIAGNOSE = 0x2
ENKF_FLAG_AUTOTUNE = 0x4
STATUS = {0: "ENKF_SUCCESS", 1: "ENKF_ERR_INVALID_ARG", 2: "ENKF_ERR_NOT_SPD", 3: "ENKF_ERR_NO_CONVERGENCE",
          4: "ENKF_ERR_HIP", 5: "ENKF_ERR_OUT_OF_MEMORY", 6: "ENKF_ERR_NOT_SUPPORTED"}
KERNEL_CLASSES = {"factor_sweep": 0, "solve_sweep": 1, "build": 2, "analysis": 3, "gram": 4,
                  "panel_update": 5, "panel_factor": 6, "residual": 7, "step1": 8,
                  "fused_sweep": 9, "localize": 10, "residual_tn": 11}


class EnkfError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}: {detail}")
        self.code = code


class SmDesc(ctypes.Structure):
    _fields_ = [("n_obs", ctypes.c_int64), ("n_ens", ctypes.c_int32), ("dtype", ctypes.c_int),
                ("algo", ctypes.c_int), ("math", ctypes.c_int), ("block", ctypes.c_int32),
                ("max_nrhs", ctypes.c_int32), ("refine_max_iter", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("flags", ctypes.c_uint32)]


class LocalDesc(ctypes.Structure):
    _fields_ = [("n_glob", ctypes.c_int64), ("n_ens", ctypes.c_int32), ("n_state", ctypes.c_int64),
                ("n_prob", ctypes.c_int64), ("tune", ctypes.c_int32)]


class SmInfo(ctypes.Structure):
    _fields_ = [("refine_iters", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("backward_error", ctypes.c_double), ("gamma_min", ctypes.c_double), ("gamma_max", ctypes.c_double),
                ("device_status", ctypes.c_int32), ("hip_error", ctypes.c_int32), ("block", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libenkf_sm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1302_3876_amd._build` "
                           "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, vp, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
    L.enkf_sm_validate_desc.argtypes = [ctypes.POINTER(SmDesc)]
    L.enkf_build_vd.argtypes = [i64, i32, ctypes.c_int, vp, i64, vp, i64, vp, vp, i64, vp, vp, i64, vp]
    L.enkf_sm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SmDesc), vp, vp, i64, vp]
    L.enkf_sm_solve.argtypes = [vp, i32, vp, i64, vp, i64, ctypes.POINTER(SmInfo)]
    L.enkf_sm_refactor.argtypes = [vp, vp, vp, i64]
    L.enkf_sm_init_block_r.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SmDesc), ctypes.POINTER(BlockR), vp, i64, vp]
    L.enkf_sm_refactor_block_r.argtypes = [vp, vp, vp, i64]
    L.enkf_sm_factor_solve.argtypes = [vp, vp, vp, i64, i32, vp, i64, vp, i64, ctypes.POINTER(SmInfo)]
    L.enkf_analysis.argtypes = [vp, i64, vp, i64, vp, i64, vp, i64]
    L.enkf_analysis_ex.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, vp, i64]
    L.enkf_localized_analysis.argtypes = [vp, i64, vp, i64, vp, i64, vp, ctypes.c_double, i64, i64, vp, i64]
    L.enkf_sm_get_info.argtypes = [vp, ctypes.POINTER(SmInfo)]
    L.enkf_sm_get_pivots.argtypes = [vp, vp, vp]
    L.enkf_sm_get_tuning.argtypes = [vp, vp, vp, ctypes.POINTER(i32)]
    L.enkf_sm_solve_noalloc.argtypes = [ctypes.POINTER(SmDesc), vp, vp, i64, i32, vp, i64, vp, i64,
                                        ctypes.POINTER(SmInfo), vp]
    L.enkf_sm_set_timing.argtypes = [vp, i32]
    L.enkf_sm_get_timing.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl)]
    L.enkf_sm_destroy.argtypes = [vp]
    L.enkf_sm_destroy.restype = None
    L.enkf_l96_forecast.argtypes = [i64, i32, vp, i64, i32, dbl, dbl, vp]
    L.enkf_l96_forecast.restype = ctypes.c_int
    L.enkf_local_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(LocalDesc), vp, vp, vp, vp]
    L.enkf_local_analysis.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, i64, vp]
    L.enkf_local_sync.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.enkf_local_get_path.argtypes = [vp, ctypes.POINTER(i32)]
    L.enkf_local_destroy.argtypes = [vp]
    L.enkf_local_destroy.restype = None
    L.enkf_mfma_peak.argtypes = [ctypes.c_int, ctypes.POINTER(dbl)]
    L.enkf_mfma_peak.restype = ctypes.c_int
    L.enkf_status_string.argtypes = [ctypes.c_int]
    L.enkf_status_string.restype = ctypes.c_char_p
    L.enkf_last_error_message.argtypes = []
    L.enkf_last_error_message.restype = ctypes.c_char_p
    for name in ("enkf_sm_validate_desc", "enkf_build_vd", "enkf_sm_init", "enkf_sm_init_block_r", "enkf_sm_refactor",
                 "enkf_sm_refactor_block_r", "enkf_sm_factor_solve", "enkf_sm_solve", "enkf_analysis",
                 "enkf_analysis_ex", "enkf_localized_analysis", "enkf_sm_get_info", "enkf_sm_get_pivots", "enkf_sm_get_tuning", "enkf_sm_solve_noalloc", "enkf_sm_set_timing", "enkf_sm_get_timing",
                 "enkf_local_init", "enkf_local_analysis", "enkf_local_sync", "enkf_local_get_path"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions(path: str = HEADER):
    """Names of the functions declared in a header of include/."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(enkf_[a-z0-9_]+)\s*\(", text)))


def _check(code: int, where: str):
    if code != 0:
        raise EnkfError(code, where, lib().enkf_last_error_message().decode())


# ------------------------------------------------------------------ tensors
def _torch():
    import torch
    return torch


def colmajor(rows: int, cols: int, dtype=None, device="cuda", fill=None):
    """Allocate a column-major (rows x cols) tensor (stride(0) == 1)."""
    torch = _torch()
    dtype = dtype or torch.float64
    t = torch.empty((cols, rows), dtype=dtype, device=device).t()
    if fill is not None:
        t.fill_(fill)
    return t


def to_colmajor(a, dtype=None, device="cuda"):
    """Copy an array/tensor into a new column-major device tensor."""
    torch = _torch()
    src = torch.as_tensor(a)
    if src.ndim == 1:
        src = src[:, None]
    out = colmajor(src.shape[0], src.shape[1], dtype or src.dtype, device)
    out.copy_(src)
    return out


def _mat(t, name, dtype_code=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.ndim != 2:
        raise ValueError(f"{name} must be 2-D (column-major)")
    if t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    if dtype_code is not None:
        want = torch.float64 if dtype_code == ENKF_F64 else torch.float32
        if t.dtype != want:
            raise TypeError(f"{name} must be {want}")
    ld = t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)
    return ctypes.c_void_p(t.data_ptr()), ld


def _vec(t, name, dtype):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.ndim != 1 or not t.is_contiguous() or t.dtype != dtype:
        raise TypeError(f"{name} must be a contiguous 1-D CUDA tensor of {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return ENKF_F64
    if t.dtype == torch.float32:
        return ENKF_F32
    raise TypeError("storage must be float64 or float32")


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ ABI calls
def enkf_sm_validate_desc(desc: SmDesc) -> int:
    return lib().enkf_sm_validate_desc(ctypes.byref(desc))


def enkf_build_vd(XB, obs_idx, y, E, V=None, D=None):
    """V = H S and D = Y - H X^B from the ensemble (see enkf_build_vd)."""
    torch = _torch()
    dt = _dtype_code(XB)
    pXB, ldx = _mat(XB, "XB", dt)
    n_state, N = XB.shape
    n_obs = obs_idx.shape[0]
    pE, lde = _mat(E, "E", dt)
    if V is None:
        V = colmajor(n_obs, N, XB.dtype, XB.device)
    if D is None:
        D = colmajor(n_obs, N, XB.dtype, XB.device)
    pV, ldv = _mat(V, "V", dt)
    pD, ldd = _mat(D, "D", dt)
    if ldd != ldv:
        raise ValueError("V and D must share a leading dimension")
    _check(lib().enkf_build_vd(n_state, N, dt, pXB, ldx, _vec(obs_idx, "obs_idx", torch.int64), n_obs,
                               _vec(y, "y", torch.float64), pE, lde, pV, pD, ldv, _stream()), "enkf_build_vd")
    return V, D


class BlockR(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("offsets", ctypes.c_void_p), ("blocks", ctypes.c_void_p)]


class Plan:
    """enkf_sm_init / enkf_sm_solve / enkf_analysis on one (r, V).

    With ``block_r=(offsets, blocks)`` (numpy int64 host offsets, FP64 device
    tensor of the packed column-major blocks) R is block diagonal and r is
    ignored (enkf_sm_init_block_r)."""

    def __init__(self, r, V, algo: str = "plain", math: Optional[str] = None, block: int = 0, max_nrhs: int = 0,
                 refine_max_iter: int = 0, refine_tol: float = 0.0, pivot: bool = False, block_r=None,
                 diagnose: bool = False, autotune: bool = False):
        torch = _torch()
        self.dtype = _dtype_code(V)
        if math is None:
            math = "f64" if self.dtype == ENKF_F64 else "f32"
        pV, ldv = _mat(V, "V", self.dtype)
        n, N = V.shape
        self.desc = SmDesc(n, N, self.dtype, ENKF_SM_PLAIN if algo == "plain" else ENKF_SM_BLOCKED, MATH[math],
                           block, max_nrhs, refine_max_iter, refine_tol,
                           (ENKF_FLAG_PIVOT if pivot else 0) | (ENKF_FLAG_DIAGNOSE if diagnose else 0)
                           | (ENKF_FLAG_AUTOTUNE if autotune else 0))
        self._r, self._V = r, V  # borrowed by the plan until close()
        self._handle = ctypes.c_void_p()
        self.n_obs, self.n_ens = n, N
        if block_r is not None:
            import numpy as np
            off = np.ascontiguousarray(block_r[0], dtype=np.int64)
            blocks = block_r[1]
            pb = _vec(blocks, "blocks", torch.float64)
            self._block_r = (off, blocks)
            R = BlockR(len(off) - 1, ctypes.c_void_p(off.ctypes.data), pb)
            _check(lib().enkf_sm_init_block_r(ctypes.byref(self._handle), ctypes.byref(self.desc), ctypes.byref(R),
                                              pV, ldv, _stream()), "enkf_sm_init_block_r")
            return
        _check(lib().enkf_sm_init(ctypes.byref(self._handle), ctypes.byref(self.desc),
                                  _vec(r, "r", torch.float64), pV, ldv, _stream()), "enkf_sm_init")

    def refactor_block_r(self, blocks, V):
        """New block values (same structure) and V (enkf_sm_refactor_block_r)."""
        torch = _torch()
        pV, ldv = _mat(V, "V", self.dtype)
        _check(lib().enkf_sm_refactor_block_r(self._handle, _vec(blocks, "blocks", torch.float64), pV, ldv),
               "enkf_sm_refactor_block_r")
        self._block_r = (self._block_r[0], blocks)
        self._V = V

    def refactor(self, r, V):
        """New (r, V) of the same shape: recompute the factor in the same
        workspace (enkf_sm_refactor)."""
        torch = _torch()
        pV, ldv = _mat(V, "V", self.dtype)
        if tuple(V.shape) != (self.n_obs, self.n_ens):
            raise ValueError("refactor: V shape differs from the plan's")
        _check(lib().enkf_sm_refactor(self._handle, _vec(r, "r", torch.float64), pV, ldv), "enkf_sm_refactor")
        self._r, self._V = r, V

    def solve(self, D, Z=None, info: bool = False):
        """Z = (R + V V^T)^{-1} D (enkf_sm_solve)."""
        pD, ldd = _mat(D, "D", self.dtype)
        if Z is None:
            Z = colmajor(D.shape[0], D.shape[1], D.dtype, D.device)
        pZ, ldz = _mat(Z, "Z", self.dtype)
        inf = SmInfo() if info else None
        _check(lib().enkf_sm_solve(self._handle, D.shape[1], pD, ldd, pZ, ldz,
                                   ctypes.byref(inf) if info else None), "enkf_sm_solve")
        return (Z, inf.as_dict()) if info else Z

    def factor_solve(self, r, V, D, Z=None, info: bool = False):
        """refactor(r, V) and solve(D) in one level loop (enkf_sm_factor_solve)."""
        torch = _torch()
        pV, ldv = _mat(V, "V", self.dtype)
        if tuple(V.shape) != (self.n_obs, self.n_ens):
            raise ValueError("factor_solve: V shape differs from the plan's")
        pD, ldd = _mat(D, "D", self.dtype)
        if Z is None:
            Z = colmajor(D.shape[0], D.shape[1], D.dtype, D.device)
        pZ, ldz = _mat(Z, "Z", self.dtype)
        inf = SmInfo() if info else None
        _check(lib().enkf_sm_factor_solve(self._handle, _vec(r, "r", torch.float64), pV, ldv, D.shape[1], pD, ldd,
                                          pZ, ldz, ctypes.byref(inf) if info else None), "enkf_sm_factor_solve")
        self._r, self._V = r, V
        return (Z, inf.as_dict()) if info else Z

    def analysis(self, XB, Z, XA=None):
        """X^A = X^B + S V^T Z (enkf_analysis)."""
        pXB, ldx = _mat(XB, "XB", self.dtype)
        pZ, ldz = _mat(Z, "Z", self.dtype)
        if XA is None:
            XA = colmajor(XB.shape[0], XB.shape[1], XB.dtype, XB.device)
        pXA, ldxa = _mat(XA, "XA", self.dtype)
        _check(lib().enkf_analysis(self._handle, XB.shape[0], pXB, ldx, pZ, ldz, pXA, ldxa), "enkf_analysis")
        return XA

    def analysis_ex(self, XB, Z, XA=None, math: str = "f32"):
        """X^A = X^B + S V^T Z with X^B/X^A in their own type and the product
        on `math` (enkf_analysis_ex)."""
        xdt = _dtype_code(XB)
        pXB, ldx = _mat(XB, "XB", xdt)
        pZ, ldz = _mat(Z, "Z", self.dtype)
        if XA is None:
            XA = colmajor(XB.shape[0], XB.shape[1], XB.dtype, XB.device)
        pXA, ldxa = _mat(XA, "XA", xdt)
        _check(lib().enkf_analysis_ex(self._handle, XB.shape[0], xdt, MATH[math], pXB, ldx, pZ, ldz, pXA, ldxa),
               "enkf_analysis_ex")
        return XA

    def localized_analysis(self, XB, Z, obs_loc, length: float, radius: int = -1, ring: int = 0, XA=None):
        """X^A = X^B + (Delta o (S V^T)) Z with the impact factors
        exp(-d/length) (enkf_localized_analysis); obs_loc: int64 device
        tensor of the observations' state indices."""
        torch = _torch()
        pXB, ldx = _mat(XB, "XB", self.dtype)
        pZ, ldz = _mat(Z, "Z", self.dtype)
        if XA is None:
            XA = colmajor(XB.shape[0], XB.shape[1], XB.dtype, XB.device)
        pXA, ldxa = _mat(XA, "XA", self.dtype)
        pl = _vec(obs_loc, "obs_loc", torch.int64)
        if obs_loc.shape[0] != self.n_obs:
            raise ValueError("localized_analysis: obs_loc needs one entry per observation")
        _check(lib().enkf_localized_analysis(self._handle, XB.shape[0], pXB, ldx, pZ, ldz, pl, float(length),
                                             int(radius), int(ring), pXA, ldxa), "enkf_localized_analysis")
        return XA

    def info(self):
        inf = SmInfo()
        _check(lib().enkf_sm_get_info(self._handle, ctypes.byref(inf)), "enkf_sm_get_info")
        return inf.as_dict()

    def tuning(self):
        """{panel width: ms of one factorisation + solve} measured by
        ENKF_FLAG_AUTOTUNE at init (empty if the plan did not tune)."""
        import numpy as np
        wd = np.zeros(4, dtype=np.int32)
        ms = np.zeros(4, dtype=np.float64)
        cnt = ctypes.c_int32(0)
        _check(lib().enkf_sm_get_tuning(self._handle, ctypes.c_void_p(wd.ctypes.data), ctypes.c_void_p(ms.ctypes.data),
                                        ctypes.byref(cnt)), "enkf_sm_get_tuning")
        return {int(wd[i]): float(ms[i]) for i in range(cnt.value)}

    def pivots(self):
        import numpy as np
        g = np.zeros(self.n_ens, dtype=np.float64)
        p = np.zeros(self.n_ens, dtype=np.int32)
        _check(lib().enkf_sm_get_pivots(self._handle, ctypes.c_void_p(g.ctypes.data), ctypes.c_void_p(p.ctypes.data)),
               "enkf_sm_get_pivots")
        return g, p

    def set_timing(self, enable: bool):
        _check(lib().enkf_sm_set_timing(self._handle, 1 if enable else 0), "enkf_sm_set_timing")

    def timing(self, kernel_class: str):
        ms, nl, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().enkf_sm_get_timing(self._handle, KERNEL_CLASSES[kernel_class], ctypes.byref(ms), ctypes.byref(nl),
                                        ctypes.byref(by), ctypes.byref(fl)), "enkf_sm_get_timing")
        return {"ms": ms.value, "launches": nl.value, "bytes": by.value, "flops": fl.value}

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib().enkf_sm_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def enkf_sm_init(r, V, **kw) -> Plan:
    return Plan(r, V, **kw)


def enkf_sm_solve(plan: Plan, D, Z=None, info: bool = False):
    return plan.solve(D, Z, info)


def enkf_analysis(plan: Plan, XB, Z, XA=None):
    return plan.analysis(XB, Z, XA)


def enkf_sm_solve_noalloc(r, V, D, Z=None, algo: str = "plain", math: Optional[str] = None, block: int = 0,
                          refine_max_iter: int = 0, refine_tol: float = 0.0, info: bool = False):
    """Factor and solve in one call with the workspace in the library's
    static device scratch: no device allocation (enkf_sm_solve_noalloc).
    Returns Z (and the info dict when info=True)."""
    torch = _torch()
    dt = _dtype_code(V)
    if math is None:
        math = "f64" if dt == ENKF_F64 else "f32"
    pV, ldv = _mat(V, "V", dt)
    pD, ldd = _mat(D, "D", dt)
    if Z is None:
        Z = colmajor(D.shape[0], D.shape[1], D.dtype, D.device)
    pZ, ldz = _mat(Z, "Z", dt)
    n, N = V.shape
    desc = SmDesc(n, N, dt, ENKF_SM_PLAIN if algo == "plain" else ENKF_SM_BLOCKED, MATH[math], block,
                  max(D.shape[1], 1) if D.shape[1] > N else 0, refine_max_iter, refine_tol, 0)
    inf = SmInfo() if info else None
    _check(lib().enkf_sm_solve_noalloc(ctypes.byref(desc), _vec(r, "r", torch.float64), pV, ldv, D.shape[1], pD, ldd,
                                       pZ, ldz, ctypes.byref(inf) if info else None, _stream()),
           "enkf_sm_solve_noalloc")
    return (Z, inf.as_dict()) if info else Z


LOCAL_TUNE = {"default": 0, "time": 1, "stream": 2, "prefix": 3}
LOCAL_PATH = {0: "stream", 1: "prefix"}


class LocalPlan:
    """Batched localized analyses (enkf_local_init / enkf_local_analysis).
    tune: True / "time" (time both paths on the first call), False /
    "default", "stream" or "prefix" (enkf_local.h, ENKF_LOCAL_TUNE_*)."""

    def __init__(self, n_glob: int, n_ens: int, n_state: int, win_start, win_len, state_idx, tune=True):
        import numpy as np
        ws = np.ascontiguousarray(win_start, dtype=np.int64)
        wl = np.ascontiguousarray(win_len, dtype=np.int64)
        si = np.ascontiguousarray(state_idx, dtype=np.int64)
        self.n_prob, self.n_ens = ws.shape[0], n_ens
        code = LOCAL_TUNE[tune] if isinstance(tune, str) else (1 if tune else 0)
        self.desc = LocalDesc(n_glob, n_ens, n_state, self.n_prob, code)
        self._handle = ctypes.c_void_p()
        _check(lib().enkf_local_init(ctypes.byref(self._handle), ctypes.byref(self.desc),
                                     ctypes.c_void_p(ws.ctypes.data), ctypes.c_void_p(wl.ctypes.data),
                                     ctypes.c_void_p(si.ctypes.data), _stream()), "enkf_local_init")

    def analysis(self, r, V, D, XB, XA=None, gamma=None):
        """Every local analysis in one launch; returns XA (n_prob x N)."""
        torch = _torch()
        pV, ldv = _mat(V, "V", ENKF_F32)
        pD, ldd = _mat(D, "D", ENKF_F32)
        if ldd != ldv:
            raise ValueError("V and D must share a leading dimension")
        pXB, ldx = _mat(XB, "XB", ENKF_F32)
        if XA is None:
            XA = colmajor(self.n_prob, self.n_ens, torch.float32, V.device)
        pXA, ldxa = _mat(XA, "XA", ENKF_F32)
        pg = None
        if gamma is not None:
            pg, ldg = _mat(gamma, "gamma", ENKF_F64)
            if ldg != self.n_prob:
                raise ValueError("gamma must have leading dimension n_prob")
        _check(lib().enkf_local_analysis(self._handle, _vec(r, "r", torch.float64), pV, pD, ldv, pXB, ldx, pXA, ldxa,
                                         pg), "enkf_local_analysis")
        return XA

    def sync(self):
        kc, nb, path = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().enkf_local_sync(self._handle, ctypes.byref(kc), ctypes.byref(nb)), "enkf_local_sync")
        _check(lib().enkf_local_get_path(self._handle, ctypes.byref(path)), "enkf_local_get_path")
        return {"rows_per_stage": kc.value, "blocks": nb.value, "path": LOCAL_PATH[path.value]}

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib().enkf_local_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ Lorenz-96 cycling filter
def mfma_peak(math: str = "f64") -> float:
    """Measured matrix-core throughput of the current device in TFLOP/s
    (enkf_mfma_peak); math is "f64", "f32", "bf16" or "f16"."""
    out = ctypes.c_double(0.0)
    _check(lib().enkf_mfma_peak(MATH[math], ctypes.byref(out)), "enkf_mfma_peak")
    return out.value


def l96_forecast(X, nsteps: int, F: float = 8.0, dt: float = 0.05):
    """Advance every column of the FP64 device matrix X by nsteps RK4 steps of
    the Lorenz-96 model, in place (enkf_l96_forecast)."""
    pX, ldx = _mat(X, "X", ENKF_F64)
    _check(lib().enkf_l96_forecast(X.shape[0], X.shape[1], pX, ldx, int(nsteps), float(F), float(dt), _stream()),
           "enkf_l96_forecast")
    return X


def cycle_l96(XB, obs_idx, ys, Es, r, nsteps: int, F: float = 8.0, dt: float = 0.05, localize=None,
              algo: str = "plain", block: int = 0):
    """The Lorenz-96 cycling filter on the device: per cycle c, forecast the
    ensemble XB (FP64, n_state x N, updated in place), build V and D from
    ys[c] and Es[c] (device tensors), factor and solve (enkf_sm_factor_solve)
    and update the ensemble (enkf_analysis, or enkf_localized_analysis with
    localize = (length, ring)). Yields after each cycle (forecast mean,
    analysis mean) as device tensors, so the caller can score them."""
    torch = _torch()
    n_state, N = XB.shape
    n_obs = obs_idx.shape[0]
    V = colmajor(n_obs, N, torch.float64, XB.device)
    D = colmajor(n_obs, N, torch.float64, XB.device)
    Z = colmajor(n_obs, N, torch.float64, XB.device)
    XA = colmajor(n_state, N, torch.float64, XB.device)
    plan = None
    try:
        for c in range(len(ys)):
            l96_forecast(XB, nsteps, F, dt)
            enkf_build_vd(XB, obs_idx, ys[c], Es[c], V, D)
            if plan is None:
                plan = Plan(r, V, algo=algo, block=block)
            plan.factor_solve(r, V, D, Z)
            if localize is None:
                plan.analysis(XB, Z, XA)
            else:
                plan.localized_analysis(XB, Z, obs_idx, localize[0], -1, localize[1], XA)
            fmean = XB.mean(dim=1)
            XB.copy_(XA)
            yield fmean, XA.mean(dim=1)
    finally:
        if plan is not None:
            plan.close()
