"""The seeded input generator: bit-reproducible, thread-count independent,
and its pieces checked against independent definitions."""
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_philox_matches_numpy_bit_generator():
    for key in ([1, 2], [20130214, 6], [2**64 - 1, 0]):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
        ref = bg.random_raw(8)
        got = np.concatenate([synth.philox4x64([1, 0, 0, 0], key), synth.philox4x64([2, 0, 0, 0], key)])
        assert np.array_equal(got, ref)


def test_normal_moments_and_offsets():
    z = synth.normal(11, 3, 400_000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert np.array_equal(synth.normal(11, 3, 1000, offset=123), z[123:1123])
    u = synth.uniform(11, 4, 100_000, 0.005, 0.02)
    assert u.min() >= 0.005 and u.max() < 0.02
    k = synth.randint(1, 9, 50_000, 16, 512)
    assert k.min() == 16 and k.max() == 512


def test_thread_count_independent():
    code = ("import sys; sys.path.insert(0, %r); import synth, hashlib; w = synth.c2(n_state=4096, n_ens=8); "
            "print(hashlib.sha256(w.XB.tobytes() + w.E.tobytes() + w.y.tobytes()).hexdigest())") % ROOT
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                   check=True).stdout.strip())
    assert outs[0] == outs[1]


def _l96_rhs(x, F=8.0):
    return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + F


def test_l96_tendency_and_rk4_order():
    x0 = synth.uniform(2, 1, 36, -1, 1) + 8.0
    # one RK4 step against an independent numpy RK4 using np.roll indexing
    a = synth.l96_advance(x0.copy(), 1, dt=0.01)
    k1 = _l96_rhs(x0); k2 = _l96_rhs(x0 + 0.005 * k1); k3 = _l96_rhs(x0 + 0.005 * k2); k4 = _l96_rhs(x0 + 0.01 * k3)
    b = x0 + 0.01 / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert np.allclose(a, b, rtol=0, atol=1e-14)
    # fourth-order convergence over a fixed horizon
    e = []
    ref = synth.l96_advance(x0.copy(), 320, dt=0.00125)
    for steps, dt in ((20, 0.02), (40, 0.01)):
        e.append(np.abs(synth.l96_advance(x0.copy(), steps, dt=dt) - ref).max())
    assert 10 < e[0] / e[1] < 22


def test_members_match_single_integration():
    X = np.asfortranarray(synth.normal(5, 2, 64 * 3).reshape(3, 64).T + 8.0)
    Y = synth.l96_advance_members(X.copy(order="F"), 7)
    for j in range(3):
        assert np.array_equal(Y[:, j], synth.l96_advance(np.ascontiguousarray(X[:, j]), 7))


def test_workload_shapes():
    w = synth.c1()
    assert w.XB.shape == (40, 20) and w.n_obs == 20 and np.all(w.obs_idx == np.arange(0, 40, 2))
    assert np.all(w.r == 0.01)
    w4 = synth.c4(n_prob=64)
    ln = w4.extra["win_len"]
    assert ln.min() >= 16 and ln.max() <= 512
    st = w4.extra["win_start"]
    assert np.all((w4.extra["state_idx"] - st) % 4096 == ln // 2)
