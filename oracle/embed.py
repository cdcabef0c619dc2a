"""Categorical embedding in front of TabNet and the audit view of its masks -- oracle
(test infrastructure only; only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import it).  It shares no code with the HIP path.

What it computes.  The paper's pipeline turns raw records (the UCI Adult rows carry 14
features, Sec. IV-A) into model inputs in a preprocessing stage (Sec. III-A), and every
invocation returns predictions with feature-attribution masks for auditors (Sec. III-B),
who read importance per original feature (Table IV).  The model the paper cites
embeds each categorical column: a level l of column c becomes row l of that column's
table, so a row of C raw columns becomes D = sum_c dim_c model features, continuous
columns passing through unchanged.  A mask over the D model features is read per raw
column by adding the entries of each column's features.

    embed:   x = concat_c ( X[:, c]                  if card_c == 0
                            T_c[X[:, c]]             if X[:, c] is a level in [0, card_c)
                            0 (dim_c zeros)          otherwise: not an integer, out of range, NaN )
    reduce:  m_col[:, c] = sum_{f in features of c} m[:, f]
    forward_raw = forward(params, embed(X_raw)) with both masks reduced.

The zero row for an invalid level is a reading (the paper does not say).
"""
from __future__ import annotations

import numpy as np

from .tabnet import forward


def _check_spec(cards, dims, tables):
    cards = np.asarray(cards, dtype=np.int64)
    dims = np.asarray(dims, dtype=np.int64)
    if cards.shape != dims.shape or cards.ndim != 1:
        raise ValueError("cards and dims must be 1-D arrays of equal length")
    if (cards < 0).any() or (dims < 1).any() or (dims[cards == 0] != 1).any():
        raise ValueError("cards >= 0, dims >= 1 and continuous columns have dim 1")
    need = int((cards * dims).sum())
    tables = np.asarray(tables, dtype=np.float64).reshape(-1)
    if tables.size != need:
        raise ValueError(f"tables hold {tables.size} values, the spec needs {need}")
    return cards, dims, tables


def embed(X_raw, cards, dims, tables):
    """[B, C] raw rows -> [B, sum(dims)] model features (float64)."""
    cards, dims, tables = _check_spec(cards, dims, tables)
    X_raw = np.asarray(X_raw, dtype=np.float64)
    B, C = X_raw.shape
    if C != cards.size:
        raise ValueError("X_raw has the wrong number of columns")
    out = np.zeros((B, int(dims.sum())), dtype=np.float64)
    at, base = 0, 0
    for c in range(C):
        v = X_raw[:, c]
        if cards[c] == 0:
            out[:, at] = v
        else:
            T = tables[base:base + cards[c] * dims[c]].reshape(cards[c], dims[c])
            ok = np.isfinite(v) & (v == np.floor(v)) & (v >= 0) & (v < cards[c])
            lv = np.where(ok, v, 0).astype(np.int64)
            out[:, at:at + dims[c]] = np.where(ok[:, None], T[lv], 0.0)
            base += cards[c] * dims[c]
        at += dims[c]
    return out


def reduce_columns(m, dims):
    """[..., sum(dims)] feature masks -> [..., C] per raw column (float64 sums)."""
    m = np.asarray(m, dtype=np.float64)
    dims = np.asarray(dims, dtype=np.int64)
    edges = np.concatenate([[0], np.cumsum(dims)])
    if m.shape[-1] != edges[-1]:
        raise ValueError("mask width does not match the embedding widths")
    return np.stack([m[..., edges[c]:edges[c + 1]].sum(axis=-1) for c in range(dims.size)], axis=-1)


def forward_raw(params, X_raw, cards, dims, tables, **kw):
    """(logits [B, n_out], masks_agg per raw column [B, C], masks_step per raw column [S, B, C])."""
    lo, ag, ms = forward(params, embed(X_raw, cards, dims, tables), **kw)
    return lo, reduce_columns(ag, dims), reduce_columns(ms, dims)
