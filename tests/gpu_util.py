"""Helpers shared by the GPU tests: device copies and the parity gates."""
import numpy as np

import oracle


def dev(a, dtype=None):
    import torch
    import paper_1302_3876_amd as pk
    a = np.asarray(a)
    if a.ndim == 1:
        t = torch.as_tensor(np.ascontiguousarray(a)).cuda()
        return t if dtype is None else t.to(dtype)
    return pk.to_colmajor(a, dtype=dtype or torch.float64)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def fp64_gate(r, V, D, Z_gpu, Z_or):
    """FP64 parity gate. The relative residual of the exact-arithmetic method
    is conditioning-limited (it grows with n), so the GPU must reach the FP64
    backward error bound and a residual no worse than twice the oracle's; the
    forward difference is bounded by the condition number times the
    oracle's own backward error."""
    rr_gpu = oracle.rel_residual(r, V, Z_gpu, D)
    rr_or = oracle.rel_residual(r, V, Z_or, D)
    eta = oracle.backward_error(r, V, Z_gpu, D)
    kappa = oracle.norm_w_estimate(r, V) / float(np.min(r))
    fwd = rel(Z_gpu, Z_or)
    assert eta <= 1e-12, eta
    assert rr_gpu <= max(1e-12, 2.0 * rr_or), (rr_gpu, rr_or)
    assert fwd <= max(1e-12, kappa * 1e-14), (fwd, kappa)
    return {"relres_gpu": rr_gpu, "relres_oracle": rr_or, "eta": eta, "fwd": fwd, "kappa": kappa}
