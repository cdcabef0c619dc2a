"""Per-row, pure-Python TabNet forward (test infrastructure only; tiny models).

An independent second spelling of the oracle's definition (see ``oracle.tabnet``),
written with explicit loops, ``math`` scalar functions and ``math.fsum`` sums and a
sparsemax by sorting in plain Python.  It exists to pin the vectorised oracle: the two
must agree to ~1e-12 on small models.  It follows TabNet as the paper cites it
(Sec. II-B) with the hyper-parameter roles of Sec. IV-A.
"""
from __future__ import annotations

import math
from typing import List, Sequence


def _bn1(y: float, bn: dict, c: int, eps: float) -> float:
    return float(bn["gamma"][c]) * (y - float(bn["mean"][c])) / math.sqrt(float(bn["var"][c]) + eps) \
        + float(bn["beta"][c])


def _sig(t: float) -> float:
    if t >= 0:
        return 1.0 / (1.0 + math.exp(-t))
    e = math.exp(t)
    return e / (1.0 + e)


def _layer(u: Sequence[float], lay: dict, N: int, eps: float) -> List[float]:
    W = lay["W"]
    y = []
    for o in range(2 * N):
        dot = math.fsum(float(W[o][k]) * u[k] for k in range(len(u)))
        y.append(_bn1(dot, lay["bn"], o, eps))
    return [y[c] * _sig(y[N + c]) for c in range(N)]


def _ft(params: dict, s: int, u: Sequence[float]) -> List[float]:
    cfg = params["config"]
    h = None
    for lay in list(params["shared"]) + list(params["indep"][s]):
        g = _layer(u if h is None else h, lay, cfg.N, cfg.bn_eps)
        h = g if h is None else [(hc + gc) * math.sqrt(0.5) for hc, gc in zip(h, g)]
    return h


def _sparsemax(z: Sequence[float]) -> List[float]:
    zs = sorted(z, reverse=True)
    k_star, c_star, run = 1, zs[0], []
    for k in range(1, len(zs) + 1):
        run.append(zs[k - 1])
        c = math.fsum(run)
        if 1.0 + k * zs[k - 1] > c:
            k_star, c_star = k, c
    tau = (c_star - 1.0) / k_star
    return [max(v - tau, 0.0) for v in z]


def forward_row(params: dict, xrow: Sequence[float]):
    """One row: (logits, mask_agg, [M_1..M_S]) as Python lists."""
    cfg = params["config"]
    D, n_d = cfg.D, cfg.n_d
    x = [_bn1(float(xrow[j]), params["bn_in"], j, cfg.bn_eps) for j in range(D)]
    P = [1.0] * D
    a = _ft(params, 0, x)[n_d:]
    acc = [0.0] * n_d
    agg_terms = [[] for _ in range(D)]
    masks = []
    for i in range(1, cfg.n_steps + 1):
        att = params["att"][i - 1]
        z = []
        for j in range(D):
            dot = math.fsum(float(att["W"][j][k]) * a[k] for k in range(cfg.n_a))
            z.append(P[j] * _bn1(dot, att["bn"], j, cfg.bn_eps))
        M = _sparsemax(z)
        P = [P[j] * (cfg.gamma - M[j]) for j in range(D)]
        h = _ft(params, i, [M[j] * x[j] for j in range(D)])
        r = [max(v, 0.0) for v in h[:n_d]]
        a = h[n_d:]
        acc = [acc[c] + r[c] for c in range(n_d)]
        eta = math.fsum(r)
        for j in range(D):
            agg_terms[j].append(eta * M[j])
        masks.append(M)
    Wf = params["W_fin"]
    logits = [math.fsum(float(Wf[o][c]) * acc[c] for c in range(n_d)) for o in range(cfg.n_out)]
    agg = [math.fsum(t) for t in agg_terms]
    den = math.fsum(agg)
    magg = [v / den for v in agg] if den > 0 else [0.0] * D
    return logits, magg, masks
