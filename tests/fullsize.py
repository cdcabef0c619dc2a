"""Full-batch parity helpers (test infrastructure): every row of a GPU launch against the
FP64 oracle, chunk by chunk in worker processes (oracle.parallel), with per-row errors
reduced to the worst rows and the gate counts.

Per row r and oracle reference (lo, ag, ms):
  logit_abs  max_o |dlogit|                    logit_rel  max_o |dlogit| / max(max_o |lo|, 1e-2)
  agg_abs    max_d |dmasks_agg|                agg_l1     sum_d |dmasks_agg|
  step_abs   max_{i,d} |dmasks_step|           step_l1    max_i sum_d |dmasks_step[i]|
  argmax     the predictions agree (ties -> lowest index on both sides)
  margin     the oracle's top-two logit gap (context for argmax flips; n_out = 1 -> inf)
"""
from __future__ import annotations

import numpy as np

from oracle import parallel
from oracle import tabnet as oracle

METRICS = ("logit_abs", "logit_rel", "agg_abs", "agg_l1", "step_abs", "step_l1")
QUANTILES = (0.5, 0.9, 0.99, 0.999)


def row_errors(got, ref):
    lo, ag, ms = (np.asarray(a, dtype=np.float64) for a in got)
    rlo, rag, rms = ref
    dl = np.abs(lo - rlo)
    out = {
        "logit_abs": dl.max(1),
        "logit_rel": dl.max(1) / np.maximum(np.abs(rlo).max(1), 1e-2),
        "agg_abs": np.abs(ag - rag).max(1),
        "agg_l1": np.abs(ag - rag).sum(1),
        "argmax": np.argmax(lo, 1) == np.argmax(rlo, 1),
    }
    if ms.shape[0]:
        dm = np.abs(ms - rms)
        out["step_abs"] = dm.max((0, 2))
        out["step_l1"] = dm.sum(2).max(0)
    else:
        out["step_abs"] = out["step_l1"] = np.zeros(lo.shape[0])
    srt = np.sort(rlo, 1)
    out["margin"] = srt[:, -1] - srt[:, -2] if rlo.shape[1] > 1 else np.full(lo.shape[0], np.inf)
    return out


def _chunk_errors(params, X, payload):
    """Worker: for each (name, outputs, weights, acts) in the payload, the per-row errors
    of the outputs against the oracle with that operand rounding (each rounding mode is
    evaluated once per chunk)."""
    cache = {}

    def ref(key):
        if key not in cache:
            cache[key] = oracle.forward(params, X, weights=key[0], acts=key[1])
        return cache[key]

    res = {}
    for name, got, weights, acts in payload:
        if isinstance(got, OracleRounded):      # the format's own error: oracle against oracle
            got = ref((got.weights, got.acts))
        res[name] = row_errors(got, ref((weights, acts)))
    return res


class OracleRounded:
    """In place of GPU outputs: the oracle itself on operands rounded as given."""

    def __init__(self, weights, acts):
        self.weights, self.acts = weights, acts


def all_rows(params, X, fetch, checks, chunk=8192, workers=None, say=print):
    """Per-row errors over every row.  fetch(lo, hi) returns {output name: (logits,
    masks_agg, masks_step) for rows lo..hi as host arrays}; checks lists (check name,
    output name or OracleRounded(weights, acts), weights, acts) and compares the output with
    the oracle on operands rounded as (weights, acts).  Returns {check name: {metric: per-row array}}."""
    def payload(lo, hi):
        outs = fetch(lo, hi)
        return [(name, src if isinstance(src, OracleRounded) else outs[src], w, a) for name, src, w, a in checks]

    parts = {name: [] for name, _, _, _ in checks}
    n = X.shape[0]
    done = 0
    for lo, res in parallel.map_rows(_chunk_errors, params, X, chunk=chunk, workers=workers, payload=payload):
        for name, e in res.items():
            parts[name].append(e)
        done += len(next(iter(res.values()))["argmax"])
        if say and (done == n or done % (chunk * 16) == 0):
            say(f"  oracle rows {done}/{n}")
    return {name: {k: np.concatenate([p[k] for p in ps]) for k in ps[0]} for name, ps in parts.items()}


def summary(e):
    """Worst value of each metric, quantiles of the main ones, and the argmax agreement."""
    s = {m: float(e[m].max()) for m in METRICS}
    for m in ("logit_abs", "agg_l1", "step_l1", "step_abs"):
        for q in QUANTILES:
            s[f"{m}_q{q}"] = float(np.quantile(e[m], q))
    s["argmax"] = float(e["argmax"].mean())
    s["rows"] = int(e["argmax"].size)
    flips = ~e["argmax"]
    s["argmax_flips_margin_max"] = float(e["margin"][flips].max()) if flips.any() else 0.0
    return s
