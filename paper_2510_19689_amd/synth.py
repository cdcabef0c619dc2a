"""Seeded synthetic TabNet models, inputs and request streams.

This module draws random numbers and serialises them; it contains none of the
TabNet arithmetic.  Both the HIP path (through the weight file) and the FP64
oracle (through the parameter dictionary) consume what it produces, so it is
the only code the two sides share.

The paper evaluates on the IBM HR, UCI Adult and BLS tables (Sec. IV-A), which
are not available here; the generators below produce seeded stand-ins with the
same widths (HR: 35 features; Adult: 6 continuous + 8 categorical raw columns)
plus a larger scale-up workload.  The model hyper-parameters of the paper's own
deployment are n_d = n_a = 8 with three decision steps (Sec. IV-A).

Weight file ``TNW1`` (little-endian):

    offset  type        field
    0       char[4]     magic "TNW1"
    4       uint32      version (1)
    8       int32[7]    D, n_d, n_a, n_steps, n_shared, n_indep, n_out
    36      uint32      reserved (0)
    40      float64     gamma (prior relaxation)
    48      float64     bn_eps
    56      uint64      number of float32 values that follow
    64      float32[]   parameters, in this order:
        input BN: mean[D], var[D], gamma[D], beta[D]
        shared GLU layer l = 0..n_shared-1: W[2N, K_l] row-major (K_0 = D, else N), BN[2N]
        step-specific layers, pass s = 0..n_steps, layer l = 0..n_indep-1:
            W[2N, K] (K = D only when n_shared == 0 and l == 0, else N), BN[2N]
        attentive FC, step i = 1..n_steps: W[D, n_a], BN[D]
        final map W_fin[n_out, n_d]
    where N = n_d + n_a and every BN block is mean, var, gamma, beta.
"""
from __future__ import annotations

import dataclasses
import math
import struct
from typing import Dict, List, Tuple

import numpy as np

MAGIC = b"TNW1"
VERSION = 1
HEADER = struct.Struct("<4sI7iIddQ")
assert HEADER.size == 64


@dataclasses.dataclass(frozen=True)
class TabNetConfig:
    D: int
    n_d: int
    n_a: int
    n_steps: int
    n_shared: int
    n_indep: int
    n_out: int
    gamma: float
    bn_eps: float = 1e-5

    @property
    def N(self) -> int:
        return self.n_d + self.n_a


# The workloads.  "rows" is the batch the workload is quoted on.
WORKLOADS: Dict[str, dict] = {
    # HR-shaped: 26 continuous N(0,1) + 9 categorical columns (1-wide embeddings).
    "hr35": dict(cfg=TabNetConfig(D=35, n_d=8, n_a=8, n_steps=3, n_shared=2, n_indep=2,
                                   n_out=2, gamma=1.3), rows=256, data="hr"),
    # Adult-shaped: 6 log-normal continuous + 8 categorical embedded at 8..16 -> D = 108.
    "adult108": dict(cfg=TabNetConfig(D=108, n_d=32, n_a=32, n_steps=5, n_shared=2, n_indep=2,
                                       n_out=2, gamma=1.5), rows=65536, data="adult"),
    # Scale-up: 200 continuous N(0,1), 20 columns zeroed with probability 0.3.
    "wide200": dict(cfg=TabNetConfig(D=200, n_d=64, n_a=64, n_steps=7, n_shared=4, n_indep=2,
                                      n_out=3, gamma=1.3), rows=1048576, data="wide"),
    # The widest resident model of the multi-model serving mix: 512 continuous N(0,1)
    # features, 10 steps (n_shared = n_indep = 2 and 2 outputs are readings).
    "wide512": dict(cfg=TabNetConfig(D=512, n_d=64, n_a=64, n_steps=10, n_shared=2, n_indep=2,
                                      n_out=2, gamma=1.3), rows=65536, data="wide512"),
}
# Seeds: weights 1000 + k, data 2000 + k, request stream 3000 (k = 1, 2, 3, 5 in the order above).
WEIGHT_SEED = {"hr35": 1001, "adult108": 1002, "wide200": 1003, "wide512": 1005}
DATA_SEED = {"hr35": 2001, "adult108": 2002, "wide200": 2003, "wide512": 2005}
REQUEST_SEED = 3000

ADULT_EMBED_DIMS = (16, 16, 14, 14, 12, 10, 10, 10)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _bn(rng: np.random.Generator, n: int) -> Dict[str, np.ndarray]:
    # Running mean ~ N(0, 0.1^2), running variance ~ U(0.5, 2); affine gamma ~ U(0.75, 1.25),
    # beta ~ N(0, 0.1^2).
    return {
        "mean": _f32(rng.normal(0.0, 0.1, n)),
        "var": _f32(rng.uniform(0.5, 2.0, n)),
        "gamma": _f32(rng.uniform(0.75, 1.25, n)),
        "beta": _f32(rng.normal(0.0, 0.1, n)),
    }


def _xavier(rng: np.random.Generator, fan_out: int, fan_in: int) -> np.ndarray:
    lim = math.sqrt(6.0 / (fan_in + fan_out))
    return _f32(rng.uniform(-lim, lim, (fan_out, fan_in)))


def layer_in_dims(cfg: TabNetConfig) -> Tuple[List[int], List[int]]:
    """Input widths of the shared layers and of one pass's step-specific layers."""
    N = cfg.N
    sh = [cfg.D if l == 0 else N for l in range(cfg.n_shared)]
    ind = [cfg.D if (cfg.n_shared == 0 and l == 0) else N for l in range(cfg.n_indep)]
    return sh, ind


def make_params(cfg: TabNetConfig, seed: int) -> dict:
    """Draw every parameter of a TabNet model (float32 values) from one seed."""
    if cfg.n_shared + cfg.n_indep < 1:
        raise ValueError("the feature transformer needs at least one GLU layer")
    rng = _rng(seed)
    N2 = 2 * cfg.N
    sh_k, ind_k = layer_in_dims(cfg)
    p = {"config": cfg, "bn_in": _bn(rng, cfg.D)}
    p["shared"] = []
    for k in sh_k:
        W = _xavier(rng, N2, k)
        p["shared"].append({"W": W, "bn": _bn(rng, N2)})
    p["indep"] = []
    for _s in range(cfg.n_steps + 1):
        layers = []
        for k in ind_k:
            W = _xavier(rng, N2, k)
            layers.append({"W": W, "bn": _bn(rng, N2)})
        p["indep"].append(layers)
    p["att"] = []
    for _i in range(cfg.n_steps):
        W = _xavier(rng, cfg.D, cfg.n_a)
        p["att"].append({"W": W, "bn": _bn(rng, cfg.D)})
    p["W_fin"] = _xavier(rng, cfg.n_out, cfg.n_d)
    return p


def _flat_bn(b) -> List[np.ndarray]:
    return [b["mean"], b["var"], b["gamma"], b["beta"]]


def flatten(params: dict) -> np.ndarray:
    """All parameters in the weight-file order, as one float32 vector."""
    parts = _flat_bn(params["bn_in"])
    for lay in params["shared"]:
        parts += [lay["W"].ravel()] + _flat_bn(lay["bn"])
    for layers in params["indep"]:
        for lay in layers:
            parts += [lay["W"].ravel()] + _flat_bn(lay["bn"])
    for lay in params["att"]:
        parts += [lay["W"].ravel()] + _flat_bn(lay["bn"])
    parts.append(params["W_fin"].ravel())
    return np.concatenate([_f32(x).ravel() for x in parts])


def n_params(cfg: TabNetConfig) -> int:
    N, N2 = cfg.N, 2 * cfg.N
    sh_k, ind_k = layer_in_dims(cfg)
    n = 4 * cfg.D
    n += sum(N2 * k + 4 * N2 for k in sh_k)
    n += (cfg.n_steps + 1) * sum(N2 * k + 4 * N2 for k in ind_k)
    n += cfg.n_steps * (cfg.D * cfg.n_a + 4 * cfg.D)
    n += cfg.n_out * cfg.n_d
    return n


def to_bytes(params: dict) -> bytes:
    cfg: TabNetConfig = params["config"]
    flat = flatten(params)
    assert flat.size == n_params(cfg)
    head = HEADER.pack(MAGIC, VERSION, cfg.D, cfg.n_d, cfg.n_a, cfg.n_steps, cfg.n_shared,
                       cfg.n_indep, cfg.n_out, 0, float(cfg.gamma), float(cfg.bn_eps), flat.size)
    return head + flat.astype("<f4").tobytes()


def write_weights(params: dict, path: str) -> None:
    with open(path, "wb") as f:
        f.write(to_bytes(params))


def read_weights(path: str) -> dict:
    """Inverse of write_weights (used to check the file round trip)."""
    with open(path, "rb") as f:
        raw = f.read()
    if len(raw) < HEADER.size:
        raise ValueError("truncated header")
    (magic, ver, D, n_d, n_a, S, n_sh, n_ind, n_out, _r, gamma, eps, n) = HEADER.unpack_from(raw)
    if magic != MAGIC or ver != VERSION:
        raise ValueError("bad magic or version")
    cfg = TabNetConfig(D, n_d, n_a, S, n_sh, n_ind, n_out, gamma, eps)
    flat = np.frombuffer(raw, dtype="<f4", count=n, offset=HEADER.size).astype(np.float32)
    if flat.size != n_params(cfg):
        raise ValueError("parameter count mismatch")
    pos = 0

    def take(*shape):
        nonlocal pos
        cnt = int(np.prod(shape))
        out = flat[pos:pos + cnt].reshape(shape).copy()
        pos += cnt
        return out

    def take_bn(m):
        return {"mean": take(m), "var": take(m), "gamma": take(m), "beta": take(m)}

    N2 = 2 * cfg.N
    sh_k, ind_k = layer_in_dims(cfg)
    p = {"config": cfg, "bn_in": take_bn(D)}
    p["shared"] = [{"W": take(N2, k), "bn": take_bn(N2)} for k in sh_k]
    p["indep"] = [[{"W": take(N2, k), "bn": take_bn(N2)} for k in ind_k] for _ in range(S + 1)]
    p["att"] = [{"W": take(D, n_a), "bn": take_bn(D)} for _ in range(S)]
    p["W_fin"] = take(n_out, n_d)
    assert pos == flat.size
    return p


# ----------------------------------------------------------------------------- inputs

def _raw_columns(kind: str, rows: int, seed: int):
    """The raw columns of the HR- and Adult-shaped inputs, in column order: a list of
    (cardinality, width, values) with cardinality 0 for a continuous column (values are
    the float32 column) and > 0 for a categorical one (values are int64 levels and the
    column carries a float32 [cardinality, width] embedding table)."""
    rng = _rng(seed)
    cols = []
    if kind == "hr":
        # 26 continuous N(0,1); 9 categorical columns with 2..10 levels, each level
        # carrying a seeded scalar value (a 1-wide embedding of its one-hot code).
        card = rng.integers(2, 11, size=9)
        tables = [rng.standard_normal(int(c)) for c in card]
        cont = rng.standard_normal((rows, 26))
        cols += [(0, 1, _f32(cont[:, j])) for j in range(26)]
        for j in range(9):
            lv = rng.integers(0, int(card[j]), size=rows)
            cols.append((int(card[j]), 1, lv, _f32(tables[j]).reshape(-1, 1)))
        return cols
    if kind == "adult":
        # 6 log-normal(0,1) columns standardised with the distribution's own moments
        # (so a row never depends on its batch), then 8 categorical columns embedded
        # at widths 16,16,14,14,12,10,10,10; the widest vocabulary has 42 levels.
        card = np.concatenate([[42], rng.integers(2, 43, size=7)])
        tables = [rng.standard_normal((int(c), d)) for c, d in zip(card, ADULT_EMBED_DIMS)]
        mu = math.exp(0.5)
        sd = math.sqrt((math.e - 1.0) * math.e)
        cont = _f32((rng.lognormal(0.0, 1.0, (rows, 6)) - mu) / sd)
        cols += [(0, 1, cont[:, j]) for j in range(6)]
        for c, tab in zip(card, tables):
            lv = rng.integers(0, int(c), size=rows)
            cols.append((int(c), tab.shape[1], lv, _f32(tab)))
        return cols
    raise ValueError(f"input family {kind!r} has no categorical columns")


def make_inputs(kind: str, rows: int, seed: int) -> np.ndarray:
    """Seeded feature matrix X[rows, D] (float32, row-major) for one workload family.

    HR- and Adult-shaped rows are the embedded form of make_raw_inputs(kind, rows, seed):
    a categorical column contributes its level's row of its embedding table."""
    if kind in ("hr", "adult"):
        cols = _raw_columns(kind, rows, seed)
        D = sum(c[1] for c in cols)
        X = np.empty((rows, D), dtype=np.float32)
        at = 0
        for c in cols:
            if c[0] == 0:
                X[:, at] = c[2]
            else:
                X[:, at:at + c[1]] = c[3][c[2]]
            at += c[1]
        return X
    rng = _rng(seed)
    if kind == "wide":
        # 200 continuous N(0,1); 20 seeded columns have each entry zeroed with p = 0.3.
        X = rng.standard_normal((rows, 200), dtype=np.float32)
        cols = np.sort(rng.choice(200, size=20, replace=False))
        zero = rng.random((rows, 20)) < 0.3
        sub = X[:, cols]
        sub[zero] = 0.0
        X[:, cols] = sub
        return X
    if kind == "wide512":
        return rng.standard_normal((rows, 512), dtype=np.float32)
    if kind == "normal":
        raise ValueError("use make_normal_inputs for plain Gaussian inputs")
    raise ValueError(f"unknown input family {kind!r}")


def make_raw_inputs(kind: str, rows: int, seed: int):
    """The same rows as make_inputs(kind, rows, seed) before embedding.

    Returns (X_raw, cards, dims, tables): X_raw[rows, C] float32 holds the continuous
    values and, in categorical columns, the level as an exact float; cards[C] (0 for a
    continuous column), dims[C] (embedding widths, 1 for a continuous column) as int32;
    tables the categorical columns' float32 embedding tables, each [card, dim] row-major,
    concatenated in column order."""
    cols = _raw_columns(kind, rows, seed)
    C = len(cols)
    X = np.empty((rows, C), dtype=np.float32)
    cards = np.zeros(C, np.int32)
    dims = np.zeros(C, np.int32)
    tabs = []
    for j, c in enumerate(cols):
        cards[j], dims[j] = c[0], c[1]
        X[:, j] = c[2]
        if c[0] > 0:
            tabs.append(c[3].reshape(-1))
    tables = np.concatenate(tabs).astype(np.float32) if tabs else np.zeros(0, np.float32)
    return X, cards, dims, tables


def make_normal_inputs(rows: int, D: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Plain N(0, scale^2) inputs for models of any width."""
    return _f32(_rng(seed).standard_normal((rows, D)) * scale)


def workload(name: str, rows: int | None = None):
    """(params, X) of a named workload; rows defaults to the workload's batch."""
    w = WORKLOADS[name]
    params = make_params(w["cfg"], WEIGHT_SEED[name])
    X = make_inputs(w["data"], w["rows"] if rows is None else rows, DATA_SEED[name])
    return params, X


# ----------------------------------------------------------------------- request streams

def request_stream(rate_per_s: float, duration_s: float, seed: int = REQUEST_SEED,
                   max_rows: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    """Open-loop Poisson arrivals (seconds from start) and per-request row counts.

    Row counts are log-uniform over 1..max_rows: floor(exp(U(0, ln(max_rows + 1)))),
    clipped to [1, max_rows].
    """
    rng = _rng(seed)
    n_est = int(rate_per_s * duration_s * 1.5) + 64
    gaps = rng.exponential(1.0 / rate_per_s, size=n_est)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_est)) + t[-1]
        t = np.concatenate([t, more])
    t = t[t < duration_s]
    rows = np.floor(np.exp(rng.uniform(0.0, math.log(max_rows + 1), size=t.size))).astype(np.int64)
    rows = np.clip(rows, 1, max_rows)
    return t, rows
