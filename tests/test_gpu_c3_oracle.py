"""Every form that bench.py times on the mixed-precision workload, at its full
size (n = 2,097,152 observations, N = 256; V_ij = g_ij s_i / sqrt(255),
r_i ~ U(0.01, 0.1), D ~ N(0, 1)), against the FP64 oracle's Z of the same
system. Z is unique (Section 3.3, Theorem 3), so every form must reach the
same solution up to rounding amplified by the condition of W.

The oracle runs Steps 1-2 of Section 3.1 once for the module (about 3 x
10^12 long operations; tens of seconds on the host cores). Gates (residuals
and backward errors formed on the host in FP64 from the returned Z):
  FP64 forms (plain; blocked with and without FP64 refinement):
    eta <= 1e-12 and relres <= max(1e-12, 2 relres_oracle);
  mixed forms (FP32, BF16x3 or FP16x2 panels refined in FP64):
    relres <= 1e-10 (the refinement gate) and eta <= 1e-12;
  every form, element by element:
    max |Z - Z_oracle| <= kappa(W) * 2^-52 * 16 * max |Z_oracle| (FP64 forms)
    and kappa(W) * 1e-10 * max |Z_oracle| (mixed: the forward error the
    residual gate allows), kappa(W) = (max r + sigma_max(V)^2) / min r."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def c3ref():
    import time
    print("c3 oracle: generating and solving (n=2097152, N=256)", flush=True)
    t0 = time.time()
    w = synth.c3()
    Zo = oracle.sm_solve(w.r, w.V, w.D)["Z"]
    wnorm = oracle.norm_w_estimate(w.r, w.V)
    rr_or = float(np.linalg.norm(w.D - w.r[:, None] * Zo - w.V @ (w.V.T @ Zo)) / np.linalg.norm(w.D))
    print(f"c3 oracle: relres {rr_or:.3e}, ||W|| est {wnorm:.4e}, {time.time() - t0:.1f} s", flush=True)
    return {"w": w, "Zo": Zo, "wnorm": wnorm, "kappa": wnorm / float(np.min(w.r)), "rr_or": rr_or,
            "zo_max": float(np.max(np.abs(Zo)))}


# (algo, math, block, refine_max_iter, refine_tol) of each benched form
FORMS = {
    "plain_f64": ("plain", "f64", 0, 0, 0.0),
    "blocked_f64_b64": ("blocked", "f64", 64, 0, 0.0),
    "blocked_f64_b128": ("blocked", "f64", 128, 0, 0.0),
    "blocked_f64_refined_b128": ("blocked", "f64", 128, 1, 0.0),
    "mixed_f32_b64": ("blocked", "f32", 64, 10, 1e-10),
    "mixed_f32_b128": ("blocked", "f32", 128, 10, 1e-10),
    "mixed_bf16x3_b64": ("blocked", "bf16x3", 64, 16, 1e-10),
    "mixed_bf16x3_b128": ("blocked", "bf16x3", 128, 16, 1e-10),
    "mixed_f16x2_b64": ("blocked", "f16x2", 64, 16, 1e-10),
    "mixed_f16x2_b128": ("blocked", "f16x2", 128, 16, 1e-10),
}


@pytest.mark.parametrize("form", list(FORMS))
def test_c3_form_matches_oracle(c3ref, form):
    import torch
    import paper_1302_3876_amd as pk
    algo, math, block, refine, tol = FORMS[form]
    print(f"c3 full size vs oracle: {form}", flush=True)
    w = c3ref["w"]
    plan = pk.Plan(dev(w.r), dev(w.V), algo=algo, math=math, block=block, refine_max_iter=refine, refine_tol=tol)
    Z, info = plan.solve(dev(w.D), info=True)
    torch.cuda.synchronize()
    Zh = host(Z)
    del Z
    plan.close()
    torch.cuda.empty_cache()
    rho = w.D - w.r[:, None] * Zh - w.V @ (w.V.T @ Zh)     # FP64 (host BLAS)
    rn, dn, zn = np.linalg.norm(rho), np.linalg.norm(w.D), np.linalg.norm(Zh)
    rr = rn / dn
    eta = rn / (c3ref["wnorm"] * zn + dn)
    fwd = float(np.max(np.abs(Zh - c3ref["Zo"]))) / c3ref["zo_max"]
    print({"form": form, "relres": rr, "relres_oracle": c3ref["rr_or"], "eta": eta, "fwd_max": fwd,
           "kappa": c3ref["kappa"], "info": info}, flush=True)
    assert eta <= 1e-12
    if math == "f64":
        assert rr <= max(1e-12, 2.0 * c3ref["rr_or"])
        assert fwd <= c3ref["kappa"] * 16 * 2.0 ** -52
    else:
        assert rr <= 1e-10
        assert fwd <= c3ref["kappa"] * 1e-10
