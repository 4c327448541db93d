"""The allocation-free call (enkf_sm_solve_noalloc: the plan's workspace in
a static device array) against the planned calls it stands for
(enkf_sm_init + enkf_sm_factor_solve) on the same inputs: the same kernels
in the same order, so Z must match bit for bit. Two calls in a row with the
second smaller (the scratch keeps the first call's contents), for the plain
and the blocked algorithms; a captured call replayed equals the eager one;
a problem too large for the scratch is refused before any launch."""
import ctypes
import gc

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, fp64_gate, host

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


@pytest.mark.parametrize("algo,math,dtype", [("plain", "f64", "f64"), ("blocked", "f64", "f64"),
                                             ("plain", "f32", "f32"), ("blocked", "f32", "f64")])
def test_noalloc_equals_planned_calls(algo, math, dtype):
    import torch
    pk = _pk()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    kw = dict(algo=algo, math=math, block=16 if algo == "blocked" else 0)
    if dtype == "f64" and math == "f32":
        kw.update(refine_max_iter=6, refine_tol=0.0)
    for (n, N, seed) in ((40000, 48, 11), (5003, 20, 12)):     # the second call is smaller
        print(f"noalloc {algo} {math}/{dtype} n={n} N={N}", flush=True)
        r, V, D = synth.small_vd(n, N, seed=seed)
        rd, Vd, Dd = dev(r), dev(V, tdt), dev(D, tdt)
        Zn, info_n = pk.enkf_sm_solve_noalloc(rd, Vd, Dd, info=True, **kw)
        plan = pk.Plan(rd, Vd, **kw)
        Zp, info_p = plan.factor_solve(rd, Vd, Dd, info=True)
        torch.cuda.synchronize()
        plan.close()
        assert info_n["device_status"] == 0 and info_p["device_status"] == 0
        assert np.array_equal(host(Zn), host(Zp))
        assert info_n["gamma_min"] == info_p["gamma_min"] and info_n["gamma_max"] == info_p["gamma_max"]
        if dtype == "f64":
            fp64_gate(r, V, D, host(Zn), oracle.sm_solve(r, V, D)["Z"])


def test_noalloc_captured_replays_equal_eager():
    import torch
    pk = _pk()
    r, V, D = synth.small_vd(20000, 32, seed=13)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rd, Vd, Dd = dev(r), dev(V), dev(D)
        Z = pk.colmajor(20000, 32)
        pk.enkf_sm_solve_noalloc(rd, Vd, Dd, Z)
        s.synchronize()
        ze = host(Z)
        gc.collect()             # no plan of an earlier test may be freed inside the capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pk.enkf_sm_solve_noalloc(rd, Vd, Dd, Z)
        for rep in range(3):
            Z.zero_()
            g.replay()
            s.synchronize()
            assert np.array_equal(host(Z), ze), rep
            torch.cuda.synchronize()
            _ = float(Dd.abs().sum())


def test_noalloc_refuses_oversized_problem():
    import torch
    pk = _pk()
    n, N = 300000, 40     # U + Z columns: 300000 x 80 x 8 bytes > 64 MiB
    rd = torch.ones(n, dtype=torch.float64, device="cuda")
    Vd = pk.colmajor(n, N, fill=0.0)
    Dd = pk.colmajor(n, N, fill=1.0)
    with pytest.raises(pk.EnkfError) as e:
        pk.enkf_sm_solve_noalloc(rd, Vd, Dd)
    assert e.value.code == 6 and "static scratch" in str(e.value)
