"""The C-ABI library on the CPU: it loads, exports every function the headers
declare, its struct layouts match the header as a C compiler lays them out,
and the host-only validation rejects bad descriptors. No GPU call is made."""
import ctypes
import os
import subprocess
import sys

import pytest

import paper_1302_3876_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


def test_library_exports_every_declared_function():
    lib = pk.lib()
    names = [n for h in HEADERS for n in pk.header_functions(h)]
    assert "enkf_sm_init" in names and "enkf_sm_solve" in names and "enkf_analysis" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_c_compiler(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "enkf_sm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(enkf_sm_desc),"
        " offsetof(enkf_sm_desc, refine_tol), offsetof(enkf_sm_desc, flags), sizeof(enkf_sm_info),"
        " offsetof(enkf_sm_info, rel_residual), offsetof(enkf_sm_info, backward_error),"
        " offsetof(enkf_sm_info, gamma_max), offsetof(enkf_sm_info, device_status),"
        " offsetof(enkf_sm_info, hip_error), offsetof(enkf_sm_info, block)); printf(\"%zu %zu\\n\", sizeof(enkf_block_r),"
        " offsetof(enkf_block_r, blocks)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(pk.SmDesc), pk.SmDesc.refine_tol.offset, pk.SmDesc.flags.offset,
            ctypes.sizeof(pk.SmInfo), pk.SmInfo.rel_residual.offset, pk.SmInfo.backward_error.offset,
            pk.SmInfo.gamma_max.offset, pk.SmInfo.device_status.offset, pk.SmInfo.hip_error.offset,
            pk.SmInfo.block.offset,
            ctypes.sizeof(pk.BlockR), pk.BlockR.blocks.offset]
    assert [int(x) for x in got] == want


def _desc(**kw):
    d = dict(n_obs=100, n_ens=8, dtype=pk.ENKF_F64, algo=pk.ENKF_SM_PLAIN, math=pk.MATH["f64"], block=0,
             max_nrhs=0, refine_max_iter=0, refine_tol=0.0, flags=0)
    d.update(kw)
    return pk.SmDesc(**d)


def test_validate_desc_accepts_good():
    assert pk.enkf_sm_validate_desc(_desc()) == 0
    assert pk.enkf_sm_validate_desc(_desc(dtype=pk.ENKF_F32, math=pk.MATH["f32"])) == 0
    assert pk.enkf_sm_validate_desc(_desc(algo=pk.ENKF_SM_BLOCKED, block=4)) == 0
    assert pk.enkf_sm_validate_desc(_desc(n_obs=1, n_ens=1)) == 0
    assert pk.enkf_sm_validate_desc(_desc(flags=pk.ENKF_FLAG_DIAGNOSE)) == 0
    assert pk.enkf_sm_validate_desc(_desc(algo=pk.ENKF_SM_BLOCKED, flags=pk.ENKF_FLAG_DIAGNOSE)) == 0
    assert pk.enkf_sm_validate_desc(_desc(algo=pk.ENKF_SM_BLOCKED, flags=pk.ENKF_FLAG_AUTOTUNE)) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(n_obs=0), 1), (dict(n_ens=0), 1), (dict(dtype=7), 1), (dict(algo=9), 1), (dict(math=11), 1),
    (dict(flags=0x10), 1), (dict(max_nrhs=-1), 1), (dict(refine_max_iter=-2), 1), (dict(refine_tol=-1.0), 1),
    (dict(math=1), 1), (dict(block=3), 1), (dict(algo=1, block=9), 1), (dict(algo=1, block=-1), 1),
    (dict(algo=1, flags=1), 6), (dict(algo=1, dtype=1, math=0), 1),
])
def test_validate_desc_rejects_bad(kw, code):
    assert pk.enkf_sm_validate_desc(_desc(**kw)) == code
    assert len(pk.lib().enkf_last_error_message()) > 0


def test_status_strings():
    lib = pk.lib()
    for code in range(7):
        assert len(lib.enkf_status_string(code)) > 3
    assert lib.enkf_status_string(99) == b"unknown status"


def test_null_arguments_rejected_without_gpu():
    lib = pk.lib()
    h = ctypes.c_void_p()
    assert lib.enkf_sm_init(None, ctypes.byref(_desc()), None, None, 100, None) == 1
    assert lib.enkf_sm_init(ctypes.byref(h), ctypes.byref(_desc()), None, None, 100, None) == 1
    assert lib.enkf_sm_solve(None, 1, None, 1, None, 1, None) == 1
    assert lib.enkf_sm_factor_solve(None, None, None, 1, 1, None, 1, None, 1, None) == 1
    assert lib.enkf_sm_init_block_r(ctypes.byref(h), ctypes.byref(_desc()), None, None, 100, None) == 1
    assert lib.enkf_sm_refactor_block_r(None, None, None, 100) == 1
    assert lib.enkf_sm_get_tuning(None, None, None, None) == 1
    assert lib.enkf_analysis(None, 1, None, 1, None, 1, None, 1) == 1
    assert lib.enkf_build_vd(10, 1, 0, None, 10, None, 5, None, None, 5, None, None, 5, None) == 1
    assert lib.enkf_build_vd(10, 4, 0, None, 10, None, 5, None, None, 5, None, None, 5, None) == 1


def test_binding_refuses_missing_library(tmp_path):
    code = ("import sys; sys.path.insert(0, %r); import paper_1302_3876_amd as pk; pk.LIB_PATH = %r\n"
            "try:\n    pk.lib()\nexcept RuntimeError as e:\n    print('raised', e)\n") % (ROOT, str(tmp_path / "none.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True).stdout
    assert out.startswith("raised")


def test_local_init_rejects_unknown_tune_value():
    """enkf_local_init validates desc.tune (ENKF_LOCAL_TUNE_*) on the host,
    before any device call."""
    import numpy as np
    ws = np.zeros(1, dtype=np.int64)
    wl = np.ones(1, dtype=np.int64)
    si = np.zeros(1, dtype=np.int64)
    for bad in (-1, 4, 99):
        desc = pk.LocalDesc(100, 8, 100, 1, bad)
        h = ctypes.c_void_p()
        code = pk.lib().enkf_local_init(ctypes.byref(h), ctypes.byref(desc), ctypes.c_void_p(ws.ctypes.data),
                                        ctypes.c_void_p(wl.ctypes.data), ctypes.c_void_p(si.ctypes.data), None)
        assert code == 1 and not h.value
