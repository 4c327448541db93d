"""Pins of the partial-localization oracle (Section 3.1.2, eq.
localized-correction-component) against what the paper and the mathematics
fix, independent of the oracle's own arithmetic:
  * no localization (delta = 1) is the plain analysis update X^B + S V^T Z;
  * one observation: the correction is the unlocalized one scaled row by row
    by that observation's impact factor (the paper's single-data-point form
    with a diagonal scaling);
  * state points farther than the radius from every observation keep X^B;
  * the impact factor on a ring depends only on cyclic distance: shifting
    every state index and observation location permutes the rows;
  * brute force with exact rational arithmetic on a tiny case;
  * planted mistakes in the oracle source fail these pins."""
import os
import shutil
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _case(n_state=30, N=6, n_obs=12, seed=0):
    g = np.random.default_rng(seed)
    XB = g.standard_normal((n_state, N))
    V = g.standard_normal((n_obs, N)) / np.sqrt(N - 1)
    Z = g.standard_normal((n_obs, N))
    loc = np.sort(g.choice(n_state, size=n_obs, replace=False)).astype(np.int64)
    return XB, V, Z, loc


def test_no_localization_is_the_plain_analysis():
    XB, V, Z, loc = _case()
    XA = oracle.localized_analysis(XB, V, Z, loc, length=1e300)
    ref = oracle.analysis(XB, V, Z)
    assert np.allclose(XA, ref, rtol=1e-13, atol=1e-13)


def test_single_observation_scales_rows():
    XB, V, Z, loc = _case(n_obs=1)
    L, ring = 7.0, XB.shape[0]
    XA = oracle.localized_analysis(XB, V, Z, loc, length=L, ring=ring)
    dX = oracle.analysis(XB, V, Z) - XB
    i = np.arange(XB.shape[0])
    d = np.abs(i - loc[0])
    d = np.minimum(d, ring - d)
    assert np.allclose(XA - XB, np.exp(-d / L)[:, None] * dX, rtol=1e-12, atol=1e-14)


def test_rows_outside_every_radius_keep_the_background():
    XB, V, Z, _ = _case(n_state=60, n_obs=4)
    loc = np.array([10, 11, 12, 13], dtype=np.int64)
    XA = oracle.localized_analysis(XB, V, Z, loc, length=5.0, radius=6)
    far = (np.arange(60) < 4) | (np.arange(60) > 19)
    assert np.array_equal(XA[far], XB[far])
    assert not np.allclose(XA[~far], XB[~far])


def test_cyclic_shift_permutes_rows():
    XB, V, Z, loc = _case(n_state=40)
    s, ring = 13, 40
    XA = oracle.localized_analysis(XB, V, Z, loc, length=9.0, ring=ring)
    XB2 = np.roll(XB, s, axis=0)                  # row i -> i + s
    XA2 = oracle.localized_analysis(XB2, V, Z, (loc + s) % ring, length=9.0, ring=ring)
    assert np.allclose(np.roll(XA, s, axis=0), XA2, rtol=1e-12, atol=1e-13)


def test_row_range_matches_full():
    XB, V, Z, loc = _case(n_state=50)
    full = oracle.localized_analysis(XB, V, Z, loc, 6.0, 12, 50)
    part = oracle.localized_rows(XB, V, Z, loc, 6.0, 12, 50, 17, 31)
    assert np.array_equal(part, full[17:31])


def test_exact_rational_brute_force():
    # radius 0 keeps only the observations at the same index, where
    # delta = exp(0) = 1, so every sum is an exact rational.
    g = np.random.default_rng(5)
    n_state, N, n_obs = 5, 3, 4
    XB = g.integers(-4, 5, (n_state, N)).astype(float)
    V = g.integers(-3, 4, (n_obs, N)).astype(float)
    Z = g.integers(-3, 4, (n_obs, N)).astype(float)
    loc = np.array([0, 2, 2, 4], dtype=np.int64)
    XA = oracle.localized_analysis(XB, V, Z, loc, length=1.0, radius=0)
    F = Fraction
    for i in range(n_state):
        mean = sum(F(int(x)) for x in XB[i]) / N
        for l in range(N):
            acc = F(0)
            for k in range(N):
                inner = sum(F(int(V[j, k])) * F(int(Z[j, l])) for j in range(n_obs) if loc[j] == i)
                acc += (F(int(XB[i, k])) - mean) * inner
            # the sums are exact rationals; S carries the factor 1/sqrt(N-1)
            val = float(F(int(XB[i, l]))) + float(acc) / np.sqrt(N - 1)
            assert abs(XA[i, l] - val) <= 1e-13 * max(1.0, abs(val))


MUTANTS = [
    ("if (ring > 0 && ring - d < d) d = ring - d;", "if (ring > 0 && ring - d > d) d = ring - d;"),  # wrong wrap
    ("return exp(-(double)d / length);", "return exp((double)d / length);"),                          # sign
    ("inner += dl[j] * AT(V, ldv, j, k) * AT(Z, ldz, j, l);", "inner += dl[j] * AT(V, ldv, j, l) * AT(Z, ldz, j, k);"),
    ("for (int32_t k = 0; k < N; ++k) S[k] = (AT(XB, ldx, i, k) - mean) / scale;",
     "for (int32_t k = 0; k < N; ++k) S[k] = AT(XB, ldx, i, k) / scale;"),                         # dropped mean
    ("if (radius >= 0 && d > radius) return 0.0;", "if (radius >= 0 && d >= radius) return 0.0;"),
]


@pytest.mark.parametrize("before,after", MUTANTS)
def test_pins_catch_planted_mistakes(tmp_path, before, after):
    here = os.path.dirname(oracle.__file__)
    src = open(os.path.join(here, "enkf_oracle.c")).read()
    assert src.count(before) == 1
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    (mdir / "enkf_oracle.c").write_text(src.replace(before, after))
    shutil.copy(os.path.join(here, "__init__.py"), mdir / "__init__.py")
    tests = os.path.dirname(os.path.abspath(__file__))
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(1, %r); sys.path.insert(2, %r)\n"
        "import test_oracle_localization as t\n"
        "bad = 0\n"
        "for f in (t.test_no_localization_is_the_plain_analysis, t.test_single_observation_scales_rows,\n"
        "          t.test_rows_outside_every_radius_keep_the_background, t.test_cyclic_shift_permutes_rows,\n"
        "          t.test_exact_rational_brute_force):\n"
        "    try:\n        f()\n    except AssertionError:\n        bad += 1\n"
        "print(bad)\n"
    ) % (str(tmp_path), os.path.dirname(here), tests)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    assert int(res.stdout.strip().splitlines()[-1]) >= 1
