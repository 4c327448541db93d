"""Pins of the oracle's Lorenz-96 RK4 forecast and cycling filter: the
equilibrium x = F, fourth-order convergence against an independent adaptive
integrator (scipy DOP853), cyclic-shift equivariance, and the filter's
analysis beating its forecast on a consistent ensemble."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth


def _rhs(t, x, F=8.0):
    return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + F


def test_equilibrium_is_fixed():
    x = np.full(40, 8.0)
    assert np.array_equal(oracle.l96_forecast(x, 50)[:, 0], x)


def test_fourth_order_against_dop853():
    g = np.random.default_rng(1)
    x0 = 8.0 + g.standard_normal(40)
    T = 0.4
    ref = solve_ivp(_rhs, (0, T), x0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    e1 = np.abs(oracle.l96_forecast(x0, 16, dt=T / 16)[:, 0] - ref).max()
    e2 = np.abs(oracle.l96_forecast(x0, 32, dt=T / 32)[:, 0] - ref).max()
    assert e1 < 0.05
    assert 12.0 < e1 / e2 < 20.0          # error ratio 2^4 for RK4


def test_cyclic_shift_equivariance():
    g = np.random.default_rng(2)
    X = 8.0 + g.standard_normal((30, 3))
    a = oracle.l96_forecast(X, 10)
    b = oracle.l96_forecast(np.roll(X, 7, axis=0), 10)
    assert np.allclose(np.roll(a, 7, axis=0), b, rtol=0, atol=1e-13)


def test_cycling_filter_reduces_error():
    n, N, cycles, nsteps = 40, 40, 6, 5
    truth = 8.0 + synth.normal(5, 1, n)
    truth = synth.l96_advance(np.ascontiguousarray(truth), 500)
    g = np.random.default_rng(3)
    XB = np.asfortranarray(truth[:, None] + 0.5 * g.standard_normal((n, N)))
    obs = np.arange(n, dtype=np.int64)
    r = np.full(n, 0.01)
    truths, ys, Es = [], [], []
    t = truth.copy()
    for c in range(cycles):
        t = synth.l96_advance(t, nsteps)
        truths.append(t.copy())
        ys.append(t + 0.1 * g.standard_normal(n))
        Es.append(np.asfortranarray(0.1 * g.standard_normal((n, N))))
    _, rf, ra = oracle.cycle_l96(XB, obs, ys, Es, r, nsteps, truths=truths)
    assert all(a < f for a, f in zip(ra, rf))
    assert ra[-1] < 0.1
