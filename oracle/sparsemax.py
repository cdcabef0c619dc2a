"""Sparsemax references in float64 (test infrastructure; never on the product path).

TabNet's attentive transformer turns its scores into a feature-selection mask with
sparsemax, and the paper relies on exactly that deterministic mask for audit
(Sec. II-B cites TabNet's sequential attention and feature masks; Sec. V-C states
that the masks come out of the forward pass through sparsemax).  Sparsemax is the
Euclidean projection of a score vector z onto the probability simplex
(Martins & Astudillo, ICML 2016):

    sparsemax(z) = argmin_{p >= 0, sum(p) = 1} ||p - z||^2  =  max(z - tau, 0)

with the threshold tau fixed by sum(max(z - tau, 0)) = 1.

Three independent routes to tau are given so that each can pin the others:
  * ``sparsemax``          -- the sort-based closed form (the definition used by the oracle);
  * ``sparsemax_support``  -- enumerate every candidate support and keep the one that
                              satisfies the optimality (KKT) conditions; tiny inputs only;
  * ``sparsemax_bisect``   -- bisection on the monotone function sum(max(z - tau, 0)).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def sparsemax(z: np.ndarray) -> np.ndarray:
    """Row-wise sparsemax of a 1-D or 2-D float array, computed in float64.

    Closed form: sort descending z_(1) >= ... >= z_(K); with c_k = sum_{j<=k} z_(j),
    the support size is k* = max{k : 1 + k z_(k) > c_k}; tau = (c_{k*} - 1) / k*.
    """
    z = np.asarray(z, dtype=np.float64)
    one_d = z.ndim == 1
    Z = z[None, :] if one_d else z
    K = Z.shape[1]
    zs = -np.sort(-Z, axis=1)                       # descending
    c = np.cumsum(zs, axis=1)
    k = np.arange(1, K + 1, dtype=np.float64)[None, :]
    cond = 1.0 + k * zs > c
    kstar = K - np.argmax(cond[:, ::-1], axis=1)    # largest k with cond true (k=1 always is)
    tau = (c[np.arange(Z.shape[0]), kstar - 1] - 1.0) / kstar
    P = np.maximum(Z - tau[:, None], 0.0)
    return P[0] if one_d else P


def sparsemax_tau(z: np.ndarray) -> float:
    """Threshold tau of one vector by the sort-based closed form."""
    z = np.asarray(z, dtype=np.float64)
    zs = np.sort(z)[::-1]
    c = np.cumsum(zs)
    k = np.arange(1, z.size + 1)
    kstar = int(k[1.0 + k * zs > c].max())
    return float((c[kstar - 1] - 1.0) / kstar)


def sparsemax_support(z) -> np.ndarray:
    """Brute force over supports (K <= 12).

    For a candidate support S the stationarity condition gives tau_S = (sum_S z - 1)/|S|;
    the projection is the unique S with z_i > tau_S on S and z_j <= tau_S off S.
    Sums use math.fsum so the result is correctly rounded.
    """
    z = [float(v) for v in np.asarray(z, dtype=np.float64).ravel()]
    K = len(z)
    if K > 12:
        raise ValueError("brute force is for K <= 12")
    found = None
    for r in range(1, K + 1):
        for S in itertools.combinations(range(K), r):
            tau = (math.fsum(z[i] for i in S) - 1.0) / r
            inside = all(z[i] > tau for i in S)
            outside = all(z[j] <= tau for j in range(K) if j not in S)
            if inside and outside:
                if found is not None:
                    raise AssertionError("two supports satisfy KKT")
                found = (S, tau)
    assert found is not None, "no support satisfies KKT"
    S, tau = found
    return np.array([max(v - tau, 0.0) for v in z])


def sparsemax_bisect(z, iters: int = 200) -> np.ndarray:
    """Bisection on f(tau) = sum(max(z - tau, 0)) - 1, which is continuous and
    non-increasing, with f(max z - 1) >= 0 and f(max z) = -1."""
    z = np.asarray(z, dtype=np.float64).ravel()
    lo, hi = z.max() - 1.0, z.max()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if math.fsum(np.maximum(z - mid, 0.0)) - 1.0 > 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 0.0:
            break
    tau = 0.5 * (lo + hi)
    return np.maximum(z - tau, 0.0)
