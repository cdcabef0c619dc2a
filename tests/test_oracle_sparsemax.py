"""Pins for the oracle's sparsemax (closed forms, exact rational KKT, bisection,
invariants).  Sparsemax produces TabNet's feature masks (Sec. V-C of the paper)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle.sparsemax import sparsemax, sparsemax_bisect, sparsemax_support, sparsemax_tau


def exact_sparsemax(z):
    """Projection onto the simplex in exact rational arithmetic via the KKT conditions."""
    z = [Fraction(v) for v in z]
    K = len(z)
    for r in range(1, K + 1):
        for S in itertools.combinations(range(K), r):
            tau = (sum(z[i] for i in S) - 1) / r
            if all(z[i] > tau for i in S) and all(z[j] <= tau for j in range(K) if j not in S):
                return [max(v - tau, Fraction(0)) for v in z]
    raise AssertionError


def test_k1_is_one():
    for v in (-3.0, 0.0, 0.25, 7.5):
        assert sparsemax(np.array([v]))[0] == 1.0


def test_k2_hard_sigmoid():
    rng = np.random.default_rng(0)
    for _ in range(200):
        z1, z2 = rng.normal(0, 2, 2)
        p = sparsemax(np.array([z1, z2]))
        p1 = min(max((z1 - z2 + 1.0) / 2.0, 0.0), 1.0)
        assert abs(p[0] - p1) < 1e-15 and abs(p[1] - (1.0 - p1)) < 1e-15


def test_uniform_and_onehot():
    for K in (1, 3, 35, 108, 200):
        p = sparsemax(np.full(K, 0.3))
        np.testing.assert_allclose(p, 1.0 / K, rtol=0, atol=1e-14)
    z = np.array([0.1, 2.5, 1.5, -1.0])          # gap of exactly 1 -> one-hot
    np.testing.assert_array_equal(sparsemax(z), [0.0, 1.0, 0.0, 0.0])


def test_hand_worked_example():
    # z = (1/2, 1/5, 1/10): all three satisfy 1 + k z_(k) > c_k, so tau = (4/5 - 1)/3 = -1/15
    p = sparsemax(np.array([0.5, 0.2, 0.1]))
    np.testing.assert_allclose(p, [0.5 + 1 / 15, 0.2 + 1 / 15, 0.1 + 1 / 15], rtol=0, atol=1e-15)
    # z = (1, 1/2, -1): k=3 fails (1 - 3 = -2 < 1/2), tau = (3/2 - 1)/2 = 1/4
    p = sparsemax(np.array([1.0, 0.5, -1.0]))
    np.testing.assert_allclose(p, [0.75, 0.25, 0.0], rtol=0, atol=1e-15)


def test_exact_rational_kkt():
    rng = np.random.default_rng(1)
    for K in range(1, 8):
        for _ in range(30):
            num = rng.integers(-40, 41, size=K)
            z = [Fraction(int(n), 16) for n in num]
            ref = exact_sparsemax(z)
            got = sparsemax(np.array([float(v) for v in z]))
            for g, r in zip(got, ref):
                assert abs(g - float(r)) <= 4e-16


def test_bruteforce_and_bisection_agree():
    rng = np.random.default_rng(2)
    for K in (2, 3, 5, 8, 12):
        for scale in (0.05, 0.5, 3.0):
            z = rng.normal(0, scale, K)
            p = sparsemax(z)
            np.testing.assert_allclose(p, sparsemax_support(z), rtol=0, atol=1e-14)
            np.testing.assert_allclose(p, sparsemax_bisect(z), rtol=0, atol=1e-12)
    for K in (35, 108, 200, 512):
        z = rng.normal(0, 0.7, K)
        np.testing.assert_allclose(sparsemax(z), sparsemax_bisect(z), rtol=0, atol=1e-12)


def test_invariants():
    rng = np.random.default_rng(3)
    Z = rng.normal(0, 1.0, (64, 50))
    P = sparsemax(Z)
    assert (P >= 0).all()
    np.testing.assert_allclose(P.sum(1), 1.0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sparsemax(Z + 3.75), P, rtol=0, atol=1e-13)        # shift
    perm = rng.permutation(50)
    np.testing.assert_allclose(sparsemax(Z[:, perm]), P[:, perm], rtol=0, atol=1e-15)
    Z2 = Z + rng.normal(0, 0.1, Z.shape)                                           # non-expansive
    assert (np.linalg.norm(sparsemax(Z2) - P, axis=1) <= np.linalg.norm(Z2 - Z, axis=1) + 1e-12).all()
    # the projection is the nearest point of the simplex: no random simplex point is closer
    for r in range(8):
        q = rng.dirichlet(np.ones(50), size=200)
        d_best = np.sum((P[r] - Z[r]) ** 2)
        assert (np.sum((q - Z[r]) ** 2, axis=1) >= d_best - 1e-12).all()


def test_tau_matches_support_threshold():
    rng = np.random.default_rng(4)
    for _ in range(50):
        z = rng.normal(0, 1.0, 20)
        tau = sparsemax_tau(z)
        assert math.isclose(np.maximum(z - tau, 0).sum(), 1.0, abs_tol=1e-13)
        assert z.max() - 1.0 <= tau <= z.max() - 1.0 / z.size + 1e-15


def test_sparsemax_is_not_softmax():
    # a planted mistake of the kind the pins must catch: softmax fails the closed forms
    z = np.array([0.1, 2.5, 1.5, -1.0])
    soft = np.exp(z) / np.exp(z).sum()
    assert not np.allclose(soft, sparsemax(z), atol=1e-3)


@pytest.mark.parametrize("K", [1, 2, 7])
def test_2d_matches_rows(K):
    rng = np.random.default_rng(5)
    Z = rng.normal(0, 1, (9, K))
    P = sparsemax(Z)
    for r in range(9):
        np.testing.assert_array_equal(P[r], sparsemax(Z[r]))
