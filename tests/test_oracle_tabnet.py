"""Pins for the FP64 TabNet oracle (CPU only).

The oracle follows TabNet as the paper cites it (Sec. II-B), with the hyper-parameter
roles of Sec. IV-A and the mask outputs of Sec. III-B / Sec. V-C.  Each test below pins
it to something other than itself: library routines (torch batch norm / GLU, scipy's
logistic), closed forms of special models, invariants, and an independent per-row
pure-Python spelling.
"""
import copy
import math

import numpy as np
import pytest
import scipy.special
import torch

from oracle import scalar, tabnet
from oracle.sparsemax import sparsemax
from paper_2510_19689_amd import synth
from paper_2510_19689_amd.synth import TabNetConfig


def tiny(D=7, n_d=3, n_a=2, S=3, n_sh=2, n_ind=2, n_out=2, gamma=1.3, seed=11):
    cfg = TabNetConfig(D=D, n_d=n_d, n_a=n_a, n_steps=S, n_shared=n_sh, n_indep=n_ind,
                       n_out=n_out, gamma=gamma)
    return synth.make_params(cfg, seed)


def test_batch_norm_matches_torch():
    rng = np.random.default_rng(0)
    y = rng.normal(0, 2, (17, 9))
    bn = synth._bn(rng, 9)
    ref = torch.nn.functional.batch_norm(
        torch.tensor(y), torch.tensor(bn["mean"], dtype=torch.float64),
        torch.tensor(bn["var"], dtype=torch.float64), torch.tensor(bn["gamma"], dtype=torch.float64),
        torch.tensor(bn["beta"], dtype=torch.float64), training=False, eps=1e-5).numpy()
    np.testing.assert_allclose(tabnet.batch_norm(y, bn, 1e-5), ref, rtol=1e-14, atol=1e-14)


def test_glu_and_sigmoid_match_libraries():
    rng = np.random.default_rng(1)
    y = rng.normal(0, 5, (11, 12))
    np.testing.assert_allclose(tabnet.sigmoid(y), scipy.special.expit(y), rtol=1e-15, atol=0)
    ref = torch.nn.functional.glu(torch.tensor(y), dim=-1).numpy()
    np.testing.assert_allclose(tabnet.glu(y, 6), ref, rtol=1e-15, atol=1e-300)
    t = np.array([40.0, 0.0, -800.0])
    s = tabnet.sigmoid(t)
    assert abs(s[0] - 1.0) < 1e-17 and s[1] == 0.5 and s[2] == 0.0


@pytest.mark.parametrize("shape", [
    dict(), dict(n_sh=0, n_ind=3), dict(n_sh=3, n_ind=0), dict(n_sh=1, n_ind=1, S=1),
    dict(D=12, n_d=4, n_a=4, S=4, n_out=3, gamma=1.5)])
def test_vectorised_equals_scalar(shape):
    p = tiny(**shape)
    X = synth.make_normal_inputs(6, p["config"].D, seed=5)
    lo, ag, ms = tabnet.forward(p, X)
    for r in range(X.shape[0]):
        l1, a1, m1 = scalar.forward_row(p, X[r])
        np.testing.assert_allclose(lo[r], l1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(ag[r], a1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(ms[:, r, :], np.array(m1), rtol=1e-12, atol=1e-12)


def test_output_shapes_and_mask_invariants():
    p, X = synth.workload("hr35", rows=64)
    lo, ag, ms = tabnet.forward(p, X)
    assert lo.shape == (64, 2) and ag.shape == (64, 35) and ms.shape == (3, 64, 35)
    assert (ms >= 0).all() and (ag >= 0).all()
    np.testing.assert_allclose(ms.sum(-1), 1.0, atol=1e-13)
    np.testing.assert_allclose(ag.sum(-1), 1.0, atol=1e-13)


def test_residual_closed_form():
    """Zero value halves in every later layer: FT(u) = L_1(u) * sqrt(0.5)^(layers-1)."""
    p = tiny(n_sh=2, n_ind=2)
    cfg = p["config"]
    N = cfg.N
    layers = p["shared"] + p["indep"][0]
    for lay in layers[1:]:
        lay["W"][:N] = 0.0
        lay["bn"]["mean"][:N] = 0.0
        lay["bn"]["beta"][:N] = 0.0
    u = synth.make_normal_inputs(5, cfg.D, seed=2).astype(np.float64)
    first = tabnet.glu_layer(u, layers[0], N, cfg.bn_eps)
    got = tabnet.feature_transformer(p, 0, u)
    np.testing.assert_allclose(got, first * math.sqrt(0.5) ** (len(layers) - 1), rtol=1e-14)


def _zero_att(p, beta0=None):
    for att in p["att"]:
        att["W"][:] = 0.0
        att["bn"]["mean"][:] = 0.0
        att["bn"]["beta"][:] = 0.0
        if beta0 is not None:
            att["bn"]["beta"][0] = beta0


def test_prior_closed_form_uniform():
    """Attentive scores all zero -> every mask is 1/D, the prior is (gamma - 1/D)^i."""
    p = tiny(D=9, S=4, gamma=1.4)
    _zero_att(p)
    X = synth.make_normal_inputs(8, 9, seed=3)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    np.testing.assert_allclose(ms, 1.0 / 9, atol=1e-15)
    for i, P in enumerate(it["prior"]):
        np.testing.assert_allclose(P, (1.4 - 1.0 / 9) ** i, rtol=1e-14)
    den = ag.sum(1)
    np.testing.assert_allclose(ag[den > 0], 1.0 / 9, atol=1e-15)


def test_prior_multiplies_scores():
    """gamma = 1 and a one-hot first mask zero that feature's prior, so its score at
    step 2 is 0 (P * h, not P + h) and the remaining scores are all 0 too -> uniform."""
    p = tiny(D=6, S=2, gamma=1.0)
    _zero_att(p, beta0=10.0)
    X = synth.make_normal_inputs(4, 6, seed=4)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    np.testing.assert_array_equal(ms[0], np.eye(6)[[0] * 4])
    np.testing.assert_allclose(it["z"][1], 0.0, atol=0)
    np.testing.assert_allclose(ms[1], 1.0 / 6, atol=1e-15)


def test_prior_recurrence_from_returned_masks():
    p, X = synth.workload("hr35", rows=32)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    cfg = p["config"]
    P = np.ones_like(ms[0])
    for i in range(cfg.n_steps):
        np.testing.assert_allclose(it["prior"][i], P, rtol=1e-14)
        P = P * (cfg.gamma - ms[i])


def test_split_order_decision_first():
    """If the attention half of h is identically 0, the attentive scores are the BN shift
    alone; with a zero shift every mask is uniform even though the decision half is live."""
    p = tiny(D=8, n_d=3, n_a=2, S=3)
    cfg = p["config"]
    N, n_d = cfg.N, cfg.n_d
    for lay in p["shared"] + [l for pas in p["indep"] for l in pas]:
        lay["W"][n_d:N] = 0.0
        lay["bn"]["mean"][n_d:N] = 0.0
        lay["bn"]["beta"][n_d:N] = 0.0
    for att in p["att"]:
        att["bn"]["mean"][:] = 0.0
        att["bn"]["beta"][:] = 0.0
    X = synth.make_normal_inputs(8, 8, seed=6)
    lo, ag, ms = tabnet.forward(p, X)
    np.testing.assert_allclose(ms, 1.0 / 8, atol=1e-15)
    assert np.abs(lo).max() > 1e-3


def test_single_step_aggregate_is_the_mask():
    p = tiny(S=1)
    X = synth.make_normal_inputs(16, 7, seed=7)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    live = it["eta"][0] > 0
    assert live.any()
    np.testing.assert_allclose(ag[live], ms[0][live], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(ag[~live], 0.0)


def test_aggregate_weights_are_decision_mass():
    p, X = synth.workload("hr35", rows=16)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    agg = sum(e[:, None] * m for e, m in zip(it["eta"], ms))
    den = agg.sum(1, keepdims=True)
    np.testing.assert_allclose(ag, agg / den, rtol=1e-13)
    # eta_i is the decision mass: sum of ReLU of the decision half, so it is >= 0
    assert all((e >= 0).all() for e in it["eta"])


def test_logits_linear_in_final_map():
    p, X = synth.workload("hr35", rows=16)
    lo, ag, ms = tabnet.forward(p, X)
    q = copy.deepcopy(p)
    q["W_fin"] = q["W_fin"].astype(np.float64) * 2.5
    lo2, ag2, ms2 = tabnet.forward(q, X)
    np.testing.assert_allclose(lo2, 2.5 * lo, rtol=1e-14)
    np.testing.assert_array_equal(ag2, ag)


def test_feature_permutation_equivariance():
    p = tiny(D=9, S=3)
    X = synth.make_normal_inputs(10, 9, seed=8)
    perm = np.random.default_rng(9).permutation(9)
    q = copy.deepcopy(p)
    for k in q["bn_in"]:
        q["bn_in"][k] = q["bn_in"][k][perm]
    q["shared"][0]["W"] = q["shared"][0]["W"][:, perm]
    for att in q["att"]:
        att["W"] = att["W"][perm, :]
        for k in att["bn"]:
            att["bn"][k] = att["bn"][k][perm]
    lo, ag, ms = tabnet.forward(p, X)
    lo2, ag2, ms2 = tabnet.forward(q, X[:, perm])
    np.testing.assert_allclose(lo2, lo, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(ag2, ag[:, perm], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ms2, ms[:, :, perm], rtol=1e-12, atol=1e-14)


def test_rows_are_independent():
    p, X = synth.workload("adult108", rows=9)
    lo, ag, ms = tabnet.forward(p, X)
    for r in (0, 4, 8):
        l1, a1, m1 = tabnet.forward(p, X[r:r + 1])
        np.testing.assert_allclose(l1[0], lo[r], rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(m1[:, 0], ms[:, r], rtol=1e-13, atol=1e-15)


def test_masks_are_sparsemax_of_scores():
    p, X = synth.workload("adult108", rows=20)
    lo, ag, ms, it = tabnet.forward(p, X, internals=True)
    for i, z in enumerate(it["z"]):
        np.testing.assert_array_equal(ms[i], sparsemax(z))


def test_unrounded_options_are_identity():
    p, X = synth.workload("hr35", rows=8)
    a = tabnet.forward(p, X)
    b = tabnet.forward(p, X, weights=None, acts=None)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_int8_forward_invariants_and_attention_half_scale(monkeypatch):
    """The INT8 forward keeps the mask invariants, stays near the exact forward, and
    quantises the attentive GEMM's input over the attention half only: a decision channel
    of h, however large, must not change the attentive scores."""
    p, X = synth.workload("hr35", rows=64)
    lo, ag, ms = tabnet.forward(p, X, weights="int8", acts="int8")
    elo, eag, ems = tabnet.forward(p, X)
    np.testing.assert_allclose(ms.sum(-1), 1.0, atol=1e-12)
    np.testing.assert_allclose(ag.sum(-1), 1.0, atol=1e-12)
    assert (ms >= 0).all() and np.abs(lo - elo).max() < 0.1
    seen = []
    real = tabnet._round_acts

    def spy(u, mode):
        seen.append(u.shape[1])
        return real(u, mode)
    monkeypatch.setattr(tabnet, "_round_acts", spy)
    tabnet.forward(p, X[:2], weights="int8", acts="int8")
    cfg = p["config"]
    # per step: the attentive input has n_a columns; FT inputs have D or N columns
    assert seen.count(cfg.n_a) == cfg.n_steps
    assert set(seen) <= {cfg.n_a, cfg.D, cfg.n_d + cfg.n_a}


def test_folded_form_equals_bn_form():
    """BN(u W^T) = u (diag(s) W)^T + (beta - s mean): the folded form the rounding
    option uses reduces to the plain definition when nothing is rounded."""
    rng = np.random.default_rng(12)
    u = rng.normal(0, 1, (7, 5))
    W = rng.normal(0, 1, (4, 5))
    bn = synth._bn(rng, 4)
    s = bn["gamma"].astype(np.float64) / np.sqrt(bn["var"].astype(np.float64) + 1e-5)
    folded = u @ (W * s[:, None]).T + (bn["beta"] - s * bn["mean"])
    np.testing.assert_allclose(tabnet._fc_bn(u, W, bn, 1e-5), folded, rtol=1e-13, atol=1e-14)


def test_paper_hyperparameters_fixture(root):
    import json, os
    with open(os.path.join(root, "tests", "golden", "paper_model.json")) as f:
        g = json.load(f)
    cfg = synth.WORKLOADS["hr35"]["cfg"]
    assert (cfg.n_d, cfg.n_a, cfg.n_steps) == (g["n_d"], g["n_a"], g["n_steps"])
    assert cfg.D == g["hr_features"]
    assert synth.WORKLOADS["hr35"]["rows"] >= g["train_batch"]


def test_golden_regression(root):
    """Oracle outputs frozen by tests/golden/make_golden.py (which calls only the oracle
    and the seeded generator); guards later edits of the oracle's arithmetic."""
    import json, os
    with open(os.path.join(root, "tests", "golden", "hr35_rows4.json")) as f:
        g = json.load(f)
    p, X = synth.workload("hr35", rows=4)
    lo, ag, ms = tabnet.forward(p, X)
    np.testing.assert_allclose(lo, g["logits"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(ag, g["masks_agg"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ms, g["masks_step"], rtol=1e-12, atol=1e-14)
