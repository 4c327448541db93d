"""The analysis step captured once in a HIP graph (stream capture through
torch.cuda.graph) and replayed: the plain level loop (one launch per level)
and the blocked panel sequence, each with the V/D build and the analysis
update. Every replay, with the program's own eager work and synchronisations
between replays and new inputs copied into the captured buffers, must equal
the eager result bitwise. The plans are created on the capturing stream
(a plan's stream is fixed at init); solves without info enqueue only
kernels and device-to-device copies."""
import gc

import numpy as np
import pytest

import oracle
import synth
from gpu_util import host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("algo,n_state,N", [("plain", 40, 20), ("blocked", 4096, 48), ("plain", 65536, 24)])
def test_graph_replays_equal_eager(algo, n_state, N):
    import torch
    import paper_1302_3876_amd as pk
    print(f"graph capture {algo} n_state={n_state} N={N}", flush=True)
    if n_state == 40:
        ws = [synth.c1(), synth.c1(seed=77)]
    else:
        ws = [synth.c2(n_state=n_state, n_ens=N), synth.c2(seed=91, n_state=n_state, n_ens=N)]
    w = ws[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        XB, E = pk.to_colmajor(w.XB), pk.to_colmajor(w.E)
        obs, y, r = (torch.as_tensor(a).cuda() for a in (w.obs_idx, w.y, w.r))
        V, D = pk.enkf_build_vd(XB, obs, y, E)
        Z, XA = pk.colmajor(w.n_obs, N), pk.colmajor(w.n_state, N)
        plan = pk.Plan(r, V, algo=algo, block=16 if algo == "blocked" else 0)

        def step():
            pk.enkf_build_vd(XB, obs, y, E, V, D)
            plan.factor_solve(r, V, D, Z)
            plan.analysis(XB, Z, XA)

        def load(wk):
            XB.copy_(torch.as_tensor(wk.XB))
            E.copy_(torch.as_tensor(wk.E))
            y.copy_(torch.as_tensor(wk.y))
            r.copy_(torch.as_tensor(wk.r))

        eager = []
        for wk in ws:
            load(wk)
            step()
            eager.append((host(Z), host(XA)))
        s.synchronize()
        gc.collect()             # no plan of an earlier test may be freed inside the capture
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        for rep in range(4):
            wk = ws[rep % 2]
            load(wk)
            XA.zero_()
            Z.zero_()
            g.replay()
            s.synchronize()
            zg, xg = host(Z), host(XA)
            assert np.array_equal(zg, eager[rep % 2][0]), rep
            assert np.array_equal(xg, eager[rep % 2][1]), rep
            # eager work of the program between replays
            torch.cuda.synchronize()
            _ = (XB * 2.0).sum().item()
    plan.close()
    # and the eager result is the oracle's (FP64 gate on the increment)
    Vo, Do = oracle.build_vd(w.XB, w.obs_idx, w.y, w.E)
    XAo = oracle.analysis(w.XB, Vo, oracle.sm_solve(w.r, Vo, Do)["Z"])
    inc, inco = eager[0][1] - w.XB, XAo - w.XB
    assert np.max(np.abs(inc - inco)) <= 1e-9 * np.max(np.abs(inco))
