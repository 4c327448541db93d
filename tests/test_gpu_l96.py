"""Lorenz-96 forecast kernel and the device cycling filter (Section 4)
against the FP64 oracle, through the C ABI.

The forecast differs from the oracle only by rounding (the device may
contract products into fused multiply-adds); twenty RK4 steps of the chaotic
model amplify that by a few units, hence 1e-12. In the cycling filter each
analysis solves a system whose condition number is about
1 + n spread^2 / ((N-1) r) ~ 5e3 here (observation error 0.01, spread 5% of
the state), so the two solves differ by ~1e-12 relative, and each one-time-
unit forecast amplifies differences about five-fold (the leading Lyapunov
exponent of Lorenz-96 at F = 8 is ~1.7): after four cycles ~1e-9. The final
ensembles are compared at 1e-6 of their scale and the RMSEs at 1e-6."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _pk():
    import paper_1302_3876_amd as pk
    return pk


@pytest.mark.parametrize("n,m,steps", [(4, 1, 3), (40, 3, 20), (300, 7, 12), (1000, 64, 20), (2000, 9, 8), (4000, 4, 6),
                                         (5000, 5, 10), (8192, 2, 5)])
def test_forecast_matches_oracle(n, m, steps):
    import torch
    g = np.random.default_rng(n + m)
    X = 8.0 + g.standard_normal((n, m))
    Xd = dev(X)
    _pk().l96_forecast(Xd, steps)
    torch.cuda.synchronize()
    ref = oracle.l96_forecast(X, steps)
    assert np.allclose(host(Xd), ref, rtol=1e-12, atol=1e-12)


def test_forecast_bad_arguments():
    import torch
    pk = _pk()
    with pytest.raises(pk.EnkfError) as e:
        pk.l96_forecast(pk.colmajor(3, 2, torch.float64), 1)
    assert e.value.code == 1
    with pytest.raises(pk.EnkfError) as e:
        pk.l96_forecast(pk.colmajor(8193, 1, torch.float64), 1)
    assert e.value.code == 6


def _cycle_inputs(n, N, cycles, nsteps, seed, sd_obs):
    """Truth spun up 1000 steps; members = truth (1 + 0.05 g) (a 5%
    background error); H = I; y = truth + N(0, sd_obs^2); perturbed
    observations per member."""
    truth = synth.l96_advance(np.ascontiguousarray(8.0 + synth.normal(seed, 1, n)), 1000)
    g = np.random.default_rng(seed)
    XB = np.asfortranarray(truth[:, None] * (1.0 + 0.05 * g.standard_normal((n, N))))
    obs = np.arange(n, dtype=np.int64)
    r = np.full(n, sd_obs ** 2)
    truths, ys, Es = [], [], []
    t = truth.copy()
    for c in range(cycles):
        t = synth.l96_advance(t, nsteps)
        truths.append(t.copy())
        ys.append(t + sd_obs * g.standard_normal(n))
        Es.append(np.asfortranarray(sd_obs * g.standard_normal((n, N))))
    return XB, obs, r, truths, ys, Es


# The localized runs use an observation error comparable to the spread:
# with R = 0.01^2 and n > N the partial localization of the update lets the
# R^{-1}-sized components of Z outside the ensemble space through (the taper
# breaks the cancellation S V^T W^{-1} relies on) and the filter diverges, in
# the oracle as on the device.
# The blocked form with R = 0.01^2: the capacitance matrix M = I + V^T R^{-1} V
# has condition ~3e5; the panels apply M^{-1} through its LDL^T factor (two
# triangular products), which keeps each analysis within rounding of the
# level-by-level formula, so the chaotic forecasts (which amplify a
# difference ~600-fold over four cycles) still end within 1e-6.
@pytest.mark.parametrize("localize,algo,sd_obs,nsteps", [(False, "plain", 0.01, 20), (True, "plain", 1.0, 5),
                                                         (True, "blocked", 1.0, 5), (False, "blocked", 1.0, 5),
                                                         (False, "blocked", 0.01, 20)])
def test_cycling_filter_matches_oracle(localize, algo, sd_obs, nsteps):
    import torch
    pk = _pk()
    n, N, cycles = 200, 60, 4
    XB, obs, r, truths, ys, Es = _cycle_inputs(n, N, cycles, nsteps, seed=7, sd_obs=sd_obs)
    loc = (float(n), n) if localize else None
    XBd = dev(XB)
    rf, ra = [], []
    for fmean, amean in pk.cycle_l96(XBd, dev(obs), [dev(y) for y in ys], [dev(E) for E in Es], dev(r), nsteps,
                                     localize=loc, algo=algo):
        c = len(rf)
        rf.append(float(np.sqrt(np.mean((host(fmean) - truths[c]) ** 2))))
        ra.append(float(np.sqrt(np.mean((host(amean) - truths[c]) ** 2))))
    torch.cuda.synchronize()
    Xo, rfo, rao = oracle.cycle_l96(XB, obs, ys, Es, r, nsteps, localize=loc, truths=truths)
    assert np.abs(host(XBd) - Xo).max() <= 1e-6 * np.abs(Xo).max()
    assert np.allclose(rf, rfo, rtol=1e-6) and np.allclose(ra, rao, rtol=1e-6)
    if sd_obs < 0.1:     # observations far more accurate than the forecast
        assert all(a < f for a, f in zip(ra, rf))


@pytest.mark.slow
def test_cycle_bench_configuration_matches_oracle():
    """The configuration bench.py times for the cycling filter: n_state =
    n_obs = 1000, N = 1000, R = 0.01^2 I, 20 RK4 steps per cycle, blocked
    solve with the panel width the library picks, from the same seeded
    inputs (synth.l96_cycle_inputs); three cycles against the oracle's
    level-by-level filter."""
    import torch
    pk = _pk()
    import bench
    c = bench.CYCLE
    cycles = 3
    XB, obs, r, truths, ys, Es = synth.l96_cycle_inputs(c["n_state"], c["n_ens"], cycles, c["nsteps"], c["seed"])
    XBd = dev(XB)
    ra = []
    for _, amean in pk.cycle_l96(XBd, dev(obs), [dev(y) for y in ys], [dev(E) for E in Es], dev(r), c["nsteps"],
                                 algo="blocked"):
        ra.append(float(np.sqrt(np.mean((host(amean) - truths[len(ra)]) ** 2))))
    torch.cuda.synchronize()
    Xo, rfo, rao = oracle.cycle_l96(XB, obs, ys, Es, r, c["nsteps"], truths=truths)
    err = np.abs(host(XBd) - Xo).max() / np.abs(Xo).max()
    print({"max_rel_ensemble_diff": err, "rmse_analysis": ra, "oracle": rao}, flush=True)
    assert err <= 1e-6
    assert np.allclose(ra, rao, rtol=1e-6)
