"""Plain FP64 TabNet forward on the CPU -- the oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
module.  It shares no code with the HIP path: it reads the raw (unfolded) parameters
of a model and never sees the folded, packed or quantised weights the library builds.

What it computes.  The paper deploys TabNet (cited in Sec. I and Sec. II-B: sequential
attention whose feature masks explain each prediction) with n_d = n_a = 8 and three
decision steps (Sec. IV-A), and every invocation returns predictions together with
the feature-attribution masks (Sec. III-B), produced inside the forward pass by
sparsemax (Sec. V-C).  The paper restates none of TabNet's equations; the forward
below is the published TabNet inference pass (Arik & Pfister, AAAI 2021), with batch
norm at inference using its running statistics:

    BN(y)      = gamma * (y - mean) / sqrt(var + eps) + beta        (per channel)
    GLU(y)     = y[:, :N] * sigmoid(y[:, N:])                       (value half, gate half)
    L(u)       = GLU(BN(u W^T))                                      (one FC + BN + GLU layer)
    FT_s(u)    : h = L_1(u); for every later layer l: h = (h + L_l(h)) * sqrt(0.5)
                 where the layers are the shared ones followed by pass s's own ones.

    x = BN_in(X);  P = 1;  a = FT_0(x)[:, n_d:];  acc = 0;  agg = 0
    for i = 1..S:
        z   = P * BN_att_i(a W_att_i^T)          (attentive transformer with prior scale)
        M_i = sparsemax(z)                        (row-wise)
        P   = P * (gamma - M_i)                   (prior update with relaxation gamma)
        h   = FT_i(M_i * x)
        r   = ReLU(h[:, :n_d]);  a = h[:, n_d:]
        acc += r;  eta_i = sum_c r_c;  agg += eta_i * M_i
    logits    = acc W_fin^T
    masks_agg = agg / sum_j agg_j    (a row whose denominator is 0 stays 0)
    masks_step = [M_1, ..., M_S]

Every such reading of a point the paper leaves open is listed with the design notes.

Optional operand rounding.  ``weights``/``acts`` select how the GEMM operands are
rounded before the (exact, float64) products, to mirror a reduced-precision path:
weights in {None, "bf16", "e4m3", "int8"} act on the BN-folded weight W' = diag(s) W
with s = gamma / sqrt(var + eps) (E4M3 with one scale per output channel,
max|W'_n|/448; INT8 with one scale per output channel, max|W'_n|/127); acts in
{None, "bf16", "e4m3", "int8"} act on each GEMM input (one scale per row, max|u_r|/448
or max|u_r|/127).  The GEMM input of the attentive transformer is the attention half
a = h[:, n_d:] alone, so its row scale is taken over those channels.  The MX formats
"mxfp8", "mxfp8_e5m2", "mxfp6", "mxfp6_e3m2" and "mxfp4" (either operand) take OCP MX blocks of 32 consecutive K positions with one
power-of-two scale each (rounding.round_mx_rows), along K for both the weight rows and
the input rows; the K position of a column is its index in the GEMM input, so the
attention half a = h[:, n_d:] starts its first block at its own column 0.  The folded shift
beta - s * mean is never rounded.  With both None the computation is the definition
above, unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from .rounding import MX_ELEMENTS, round_bf16, round_e4m3, round_int8_rows, round_mx_rows, E4M3_MAX
from .sparsemax import sparsemax

SQRT_HALF = math.sqrt(0.5)


def _d(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def batch_norm(y: np.ndarray, bn: dict, eps: float) -> np.ndarray:
    """Inference batch norm with running statistics (per channel = last axis)."""
    return _d(bn["gamma"]) * (y - _d(bn["mean"])) / np.sqrt(_d(bn["var"]) + eps) + _d(bn["beta"])


def sigmoid(t: np.ndarray) -> np.ndarray:
    """Logistic function, evaluated without overflow for either sign."""
    t = np.asarray(t, dtype=np.float64)
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def glu(y: np.ndarray, N: int) -> np.ndarray:
    """Gated linear unit: first N channels are the value, last N the gate."""
    return y[:, :N] * sigmoid(y[:, N:])


def _round_acts(u: np.ndarray, mode):
    if mode is None:
        return u
    if mode == "bf16":
        return round_bf16(u)
    if mode == "e4m3":
        amax = np.max(np.abs(u), axis=1, keepdims=True)
        scale = np.where(amax > 0, amax / E4M3_MAX, 1.0)
        return round_e4m3(u / scale) * scale
    if mode == "int8":
        return round_int8_rows(u)
    if mode in MX_ELEMENTS:
        return round_mx_rows(u, mode)
    raise ValueError(mode)


def _fc_bn(u: np.ndarray, W, bn: dict, eps: float, weights=None, acts=None) -> np.ndarray:
    """BN(u W^T); with rounding enabled, the BN-folded form on rounded operands."""
    if weights is None and acts is None:
        return batch_norm(u @ _d(W).T, bn, eps)
    s = _d(bn["gamma"]) / np.sqrt(_d(bn["var"]) + eps)
    Wf = _d(W) * s[:, None]
    shift = _d(bn["beta"]) - s * _d(bn["mean"])
    if weights == "bf16":
        Wf = round_bf16(Wf)
    elif weights == "e4m3":
        amax = np.max(np.abs(Wf), axis=1, keepdims=True)
        sc = np.where(amax > 0, amax / E4M3_MAX, 1.0)
        Wf = round_e4m3(Wf / sc) * sc
    elif weights == "int8":
        Wf = round_int8_rows(Wf)
    elif weights in MX_ELEMENTS:
        Wf = round_mx_rows(Wf, weights)
    elif weights is not None:
        raise ValueError(weights)
    return _round_acts(u, acts) @ Wf.T + shift


def glu_layer(u, layer: dict, N: int, eps: float, weights=None, acts=None) -> np.ndarray:
    return glu(_fc_bn(u, layer["W"], layer["bn"], eps, weights, acts), N)


def feature_transformer(params: dict, s: int, u: np.ndarray, weights=None, acts=None) -> np.ndarray:
    """Pass s of the feature transformer: shared layers, then pass s's own layers."""
    cfg = params["config"]
    layers = list(params["shared"]) + list(params["indep"][s])
    h = None
    for lay in layers:
        g = glu_layer(u if h is None else h, lay, cfg.N, cfg.bn_eps, weights, acts)
        h = g if h is None else (h + g) * SQRT_HALF
    return h


def forward(params: dict, X, weights=None, acts=None, internals: bool = False):
    """TabNet inference on X[B, D]; returns (logits[B, n_out], masks_agg[B, D],
    masks_step[S, B, D]) in float64, plus a dict of intermediates if requested."""
    cfg = params["config"]
    X = _d(X)
    B = X.shape[0]
    n_d = cfg.n_d
    x = batch_norm(X, params["bn_in"], cfg.bn_eps)
    P = np.ones((B, cfg.D))
    a = feature_transformer(params, 0, x, weights, acts)[:, n_d:]
    acc = np.zeros((B, n_d))
    agg = np.zeros((B, cfg.D))
    masks, zs, priors, etas = [], [], [], []
    for i in range(1, cfg.n_steps + 1):
        att = params["att"][i - 1]
        z = P * _fc_bn(a, att["W"], att["bn"], cfg.bn_eps, weights, acts)
        M = sparsemax(z)
        priors.append(P)
        P = P * (cfg.gamma - M)
        h = feature_transformer(params, i, M * x, weights, acts)
        r = np.maximum(h[:, :n_d], 0.0)
        a = h[:, n_d:]
        acc = acc + r
        eta = r.sum(axis=1)
        agg = agg + eta[:, None] * M
        masks.append(M)
        zs.append(z)
        etas.append(eta)
    logits = acc @ _d(params["W_fin"]).T
    den = agg.sum(axis=1)
    safe = np.where(den > 0, den, 1.0)
    masks_agg = np.where(den[:, None] > 0, agg / safe[:, None], 0.0)
    masks_step = np.stack(masks) if masks else np.zeros((0, B, cfg.D))
    if internals:
        return logits, masks_agg, masks_step, {
            "x": x, "z": zs, "prior": priors, "eta": etas, "acc": acc, "agg": agg}
    return logits, masks_agg, masks_step
