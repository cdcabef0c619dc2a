"""Pins of the embedding / per-raw-column mask oracle (oracle/embed.py): the synthetic
generator's own embedding of the same rows, the one-hot-product form of an embedding,
closed forms of the reduction, the simplex property of reduced masks, and the reduction
of forward_raw to forward when every column is continuous."""
import numpy as np
import pytest

from oracle import embed as oe
from oracle import tabnet as ot
from paper_2510_19689_amd import synth


@pytest.mark.parametrize("kind,seed", [("adult", 2002), ("hr", 2001)])
def test_embedding_reproduces_generator(kind, seed):
    # the generator embeds with its own lookup; the oracle's must give the same rows
    X_raw, cards, dims, tables = synth.make_raw_inputs(kind, 700, seed)
    X = synth.make_inputs(kind, 700, seed)
    E = oe.embed(X_raw, cards, dims, tables)
    assert E.shape == X.shape
    np.testing.assert_array_equal(E.astype(np.float32), X)


def test_embedding_is_one_hot_product():
    rng = np.random.default_rng(3)
    cards, dims = np.array([0, 5, 0, 3]), np.array([1, 4, 1, 2])
    T1, T3 = rng.standard_normal((5, 4)), rng.standard_normal((3, 2))
    tables = np.concatenate([T1.ravel(), T3.ravel()])
    B = 50
    X = np.stack([rng.standard_normal(B), rng.integers(0, 5, B), rng.standard_normal(B),
                  rng.integers(0, 3, B)], axis=1)
    E = oe.embed(X, cards, dims, tables)
    onehot1 = (X[:, 1:2] == np.arange(5)[None]).astype(float)
    onehot3 = (X[:, 3:4] == np.arange(3)[None]).astype(float)
    np.testing.assert_array_equal(E[:, 0], X[:, 0])
    np.testing.assert_allclose(E[:, 1:5], onehot1 @ T1, rtol=0, atol=0)
    np.testing.assert_array_equal(E[:, 5], X[:, 2])
    np.testing.assert_allclose(E[:, 6:8], onehot3 @ T3, rtol=0, atol=0)
    # identity tables give the one-hot code itself: one 1 per group, at the level
    I = oe.embed(X[:, 1:2], [5], [5], np.eye(5).ravel())
    assert (I.sum(1) == 1).all() and (I.argmax(1) == X[:, 1]).all()


def test_invalid_levels_embed_to_zero():
    T = np.arange(1.0, 7.0)          # 3 levels x 2
    X = np.array([[0.0], [2.0], [-1.0], [3.0], [1.5], [np.nan], [np.inf], [1.0]])
    E = oe.embed(X, [3], [2], T)
    np.testing.assert_array_equal(E, [[1, 2], [5, 6], [0, 0], [0, 0], [0, 0], [0, 0], [0, 0], [3, 4]])
    # a continuous NaN passes through
    assert np.isnan(oe.embed(np.array([[np.nan]]), [0], [1], np.zeros(0))[0, 0])


def test_reduce_closed_form_and_totals():
    m = np.arange(1.0, 7.0)[None]
    np.testing.assert_array_equal(oe.reduce_columns(m, [1, 2, 3]), [[1, 5, 15]])
    rng = np.random.default_rng(4)
    m = rng.random((3, 9, 10))
    r = oe.reduce_columns(m, [2, 1, 4, 3])
    assert r.shape == (3, 9, 4)
    np.testing.assert_allclose(r.sum(-1), m.sum(-1), rtol=1e-14)
    with pytest.raises(ValueError):
        oe.reduce_columns(m, [2, 2])


def test_forward_raw_masks_stay_on_the_simplex():
    cfg = synth.WORKLOADS["adult108"]["cfg"]
    params = synth.make_params(cfg, synth.WEIGHT_SEED["adult108"])
    X_raw, cards, dims, tables = synth.make_raw_inputs("adult", 64, 2002)
    lo, ag, ms = oe.forward_raw(params, X_raw, cards, dims, tables)
    lo2, ag2, ms2 = ot.forward(params, oe.embed(X_raw, cards, dims, tables))
    np.testing.assert_array_equal(lo, lo2)
    assert ag.shape == (64, 14) and ms.shape == (cfg.n_steps, 64, 14)
    assert (ms >= 0).all() and (ag >= 0).all()
    np.testing.assert_allclose(ms.sum(-1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(ag.sum(-1), 1.0, rtol=1e-12)


def test_all_continuous_spec_is_plain_forward():
    cfg = synth.WORKLOADS["hr35"]["cfg"]
    params = synth.make_params(cfg, synth.WEIGHT_SEED["hr35"])
    X = synth.make_inputs("hr", 32, 2001)
    lo, ag, ms = oe.forward_raw(params, X, np.zeros(35), np.ones(35), np.zeros(0))
    lo2, ag2, ms2 = ot.forward(params, X)
    np.testing.assert_array_equal(lo, lo2)
    np.testing.assert_array_equal(ag, ag2)
    np.testing.assert_array_equal(ms, ms2)


def test_spec_validation():
    with pytest.raises(ValueError):
        oe.embed(np.zeros((1, 2)), [0, 3], [1, 2], np.zeros(5))     # tables too short
    with pytest.raises(ValueError):
        oe.embed(np.zeros((1, 1)), [0], [2], np.zeros(0))           # continuous with dim 2
    with pytest.raises(ValueError):
        oe.embed(np.zeros((1, 3)), [0, 0], [1, 1], np.zeros(0))     # wrong column count
