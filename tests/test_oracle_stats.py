"""Pins of the mask-statistics oracle (oracle/stats.py) against values fixed by the
mathematics: exact rational statistics from the standard library, closed forms and the
invariances of mean and variance."""
import statistics
from fractions import Fraction

import numpy as np
import pytest

from oracle import stats


def test_matches_exact_rational_statistics():
    # statistics.fmean / pvariance convert floats to exact fractions: an independent,
    # exactly rounded reference for small columns
    rng = np.random.default_rng(11)
    for n, D in [(1, 3), (2, 1), (5, 4), (37, 6), (200, 3)]:
        m = rng.random((n, D)).astype(np.float32)
        mean, var = stats.column_mean_var(m)
        for d in range(D):
            col = [float(v) for v in m[:, d]]
            assert mean[d] == pytest.approx(statistics.fmean(col), rel=1e-15, abs=1e-17)
            assert var[d] == pytest.approx(statistics.pvariance(col), rel=1e-12, abs=1e-17)


def test_closed_forms():
    mean, var = stats.column_mean_var([[0.0, 1.0, 0.25], [1.0, 1.0, 0.75]])
    np.testing.assert_array_equal(mean, [0.5, 1.0, 0.5])
    np.testing.assert_array_equal(var, [0.25, 0.0, 0.0625])
    # one row: mean is the row, variance 0
    mean, var = stats.column_mean_var([[0.3, 0.7]])
    np.testing.assert_array_equal(mean, [0.3, 0.7])
    np.testing.assert_array_equal(var, [0.0, 0.0])
    # k ones and n-k zeros: mean p = k/n, variance p(1-p) (Bernoulli)
    n, k = 40, 13
    col = np.zeros((n, 1))
    col[:k] = 1.0
    mean, var = stats.column_mean_var(col)
    p = Fraction(k, n)
    assert mean[0] == float(p)
    assert var[0] == pytest.approx(float(p * (1 - p)), rel=1e-15)


def test_invariances():
    rng = np.random.default_rng(12)
    m = rng.random((300, 5))
    mean, var = stats.column_mean_var(m)
    # shift: mean moves, variance does not
    m2, v2 = stats.column_mean_var(m + 1000.0)
    np.testing.assert_allclose(m2, mean + 1000.0, rtol=1e-14)
    np.testing.assert_allclose(v2, var, rtol=1e-8)
    # scale by 2 (exact): mean doubles, variance x4, bit for bit
    m3, v3 = stats.column_mean_var(2.0 * m)
    np.testing.assert_array_equal(m3, 2.0 * mean)
    np.testing.assert_array_equal(v3, 4.0 * var)
    # row order does not matter (up to rounding)
    perm = rng.permutation(300)
    m4, v4 = stats.column_mean_var(m[perm])
    np.testing.assert_allclose(m4, mean, rtol=1e-14)
    np.testing.assert_allclose(v4, var, rtol=1e-13)
    # columns are independent: a column's statistics ignore the others
    m5, v5 = stats.column_mean_var(np.ascontiguousarray(m[:, 2:3]))
    assert m5[0] == pytest.approx(mean[2], rel=1e-15) and v5[0] == pytest.approx(var[2], rel=1e-14)


def test_variance_is_mean_square_minus_square_mean():
    # E[(x - mean)^2] = E[x^2] - mean^2, computed here in exact fractions
    rng = np.random.default_rng(13)
    col = [float(v) for v in rng.random(50).astype(np.float32)]
    exact_mean = sum(Fraction(v) for v in col) / len(col)
    exact_var = sum(Fraction(v) ** 2 for v in col) / len(col) - exact_mean ** 2
    _, var = stats.column_mean_var(np.array(col)[:, None])
    assert var[0] == pytest.approx(float(exact_var), rel=1e-13)


def test_window():
    rng = np.random.default_rng(14)
    bs = [rng.random((n, 3)) for n in (4, 7, 1, 9)]
    mean, var, rows = stats.window_mean_var(bs, 2)
    assert rows == 10
    em, ev = stats.column_mean_var(np.concatenate(bs[2:]))
    np.testing.assert_array_equal(mean, em)
    np.testing.assert_array_equal(var, ev)
    mean, var, rows = stats.window_mean_var(bs, 99)
    assert rows == 21
    with pytest.raises(ValueError):
        stats.window_mean_var(bs, 0)
    with pytest.raises(ValueError):
        stats.column_mean_var(np.zeros((0, 3)))
