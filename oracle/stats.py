"""Per-feature statistics of feature-attribution masks -- oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
module; it shares no code with the HIP path.

What it computes.  The paper assesses whether TabNet's masks stay stable under load by the
variance of each feature's mask value over many served rows (Sec. IV-C, Sec. V-C: 100
random samples at peak throughput), and reports per-feature importance next to it
(Table IV).  The paper gives no formula for its stability score; the computable part is
the per-feature mean (the importance of feature d over a set of rows) and the
per-feature population variance over the same rows:

    mean_d = (1/n) sum_r m[r, d]
    var_d  = (1/n) sum_r (m[r, d] - mean_d)^2

written out here as the two-pass definition in float64.  ``window_mean_var`` is the same
statistic over the rows of the last K batches of a stream of batches.
"""
from __future__ import annotations

import numpy as np


def column_mean_var(m):
    """Per-column mean and population variance (float64, two passes) of an [n, D] array.

    n must be at least 1.  Returns (mean [D], var [D])."""
    m = np.asarray(m, dtype=np.float64)
    if m.ndim != 2 or m.shape[0] < 1:
        raise ValueError("column_mean_var needs an [n >= 1, D] array")
    n = m.shape[0]
    mean = m.sum(axis=0) / n
    dev = m - mean
    var = (dev * dev).sum(axis=0) / n
    return mean, var


def window_mean_var(batches, window: int):
    """Statistics over the rows of the last ``window`` batches of a list of [n_i, D] arrays.

    Returns (mean, var, rows)."""
    if window < 1 or not batches:
        raise ValueError("window_mean_var needs window >= 1 and at least one batch")
    rows = np.concatenate([np.asarray(b, dtype=np.float64) for b in batches[-window:]], axis=0)
    mean, var = column_mean_var(rows)
    return mean, var, rows.shape[0]
