"""GPU parity of the raw-row forward (categorical embedding gathered in the kernel, masks
per raw column) with the FP64 oracle (oracle/embed.py) and with tabnet_forward on the
embedded rows.

Gates.  The logits must equal tabnet_forward's on the embedded rows bit for bit (the kernel
sees the same FP32 features), and each raw column's mask the FP32 sum of that forward's
feature masks (|d| <= 1e-6: a sum of at most 16 values below 1).  Against the FP64 oracle
the FP32 gates of the feature-level tests apply, the mask gate times the widest column
(16 features): HR-shaped logits 1e-5 relative and masks 1e-6, Adult-shaped 1e-4 and
16 x 1e-5; BF16 logits 2e-2, aggregate-mask L1 1e-2, step-mask L1 2e-2."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import embed as oe  # noqa: E402
from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402

pytestmark = pytest.mark.gpu

KINDS = {"adult108": "adult", "hr35": "hr"}


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")


def model(name, prec, tmp_path):
    params = synth.make_params(synth.WORKLOADS[name]["cfg"], synth.WEIGHT_SEED[name])
    path = str(tmp_path / f"{name}.tnw")
    synth.write_weights(params, path)
    return params, tb.Model(path, prec)


def raw_rows(name, B, seed=None):
    return synth.make_raw_inputs(KINDS[name], B, synth.DATA_SEED[name] if seed is None else seed)


def to_np(*ts):
    torch.cuda.synchronize()
    return [None if t is None else t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "int8", "mxfp8", "mxfp8_e5m2", "mxfp6", "mxfp6_e3m2",
                                  "mxfp4"])
@pytest.mark.parametrize("name", ["adult108", "hr35"])
@pytest.mark.parametrize("B", [1, 63, 65, 1000])
def test_raw_equals_embedded_forward(name, prec, B, tmp_path):
    _say(f"case raw vs embedded {name} {prec} B={B}")
    params, m = model(name, prec, tmp_path)
    with m:
        X_raw, cards, dims, tables = raw_rows(name, B)
        X = synth.make_inputs(KINDS[name], B, synth.DATA_SEED[name])
        m.set_embeddings(cards, dims, tables)
        lo_r, ag_r, ms_r = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
        lo, ag, ms = to_np(*m.forward(torch.from_numpy(X).cuda()))
    np.testing.assert_array_equal(lo_r, lo)
    np.testing.assert_allclose(ag_r, oe.reduce_columns(ag, dims), rtol=0, atol=1e-6)
    np.testing.assert_allclose(ms_r, oe.reduce_columns(ms, dims), rtol=0, atol=1e-6)


# one model per compiled shape family: (D, n_d, n_a); then four between the families, on
# the generic kernels' raw-row twins (FP32 and BF16)
RANDOM_SHAPES = [(13, 5, 6), (30, 8, 8), (47, 4, 10), (60, 20, 12), (104, 40, 24), (205, 70, 58),
                 (150, 48, 48), (90, 20, 20), (40, 8, 40), (180, 70, 50)]


def random_spec(D, rng):
    """A random embedding of D model features: continuous columns (width 1) and categorical
    columns of 2-60 levels and width 1-24, so that columns start and end anywhere in the
    16-feature tiles; float32 tables N(0, 1)."""
    cards, dims, at = [], [], 0
    while at < D:
        if rng.random() < 0.4:
            cards.append(0)
            dims.append(1)
        else:
            dims.append(int(rng.integers(1, min(24, D - at) + 1)))
            cards.append(int(rng.integers(2, 61)))
        at += dims[-1]
    cards = np.array(cards, np.int32)
    dims = np.array(dims, np.int32)
    return cards, dims, rng.normal(0, 1, int((cards.astype(np.int64) * dims).sum())).astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("k", range(len(RANDOM_SHAPES)))
def test_random_embedding_specs(k, prec, tmp_path):
    """Random embeddings on every compiled shape family and on four generic shapes: the
    raw-row logits equal the embedded forward's bit for bit, each column's masks equal the
    FP32 sum of its features' masks (|d| <= 2e-6: at most 24 values below 1), and in FP32
    the raw forward matches the FP64 oracle (logits 1e-4 relative, masks 1e-5 times the
    widest column and the prior's growth).  A few categorical entries hold invalid levels,
    which embed to zero."""
    rng = np.random.default_rng(400 + k)
    D, n_d, n_a = RANDOM_SHAPES[k]
    cfg = synth.TabNetConfig(D=D, n_d=n_d, n_a=n_a, n_steps=int(rng.integers(1, 6)), n_shared=int(rng.integers(1, 3)),
                             n_indep=int(rng.integers(0, 3)), n_out=int(rng.integers(1, 6)),
                             gamma=float(rng.uniform(1.0, 1.8)))
    cards, dims, tables = random_spec(D, rng)
    B = int(rng.integers(1, 400))
    X_raw = np.empty((B, cards.size), np.float32)
    for c, card in enumerate(cards):
        X_raw[:, c] = rng.normal(0, 1, B) if card == 0 else rng.integers(0, card, B)
    cat = np.nonzero(cards)[0]
    if cat.size and B > 3:
        X_raw[0, cat[0]], X_raw[1, cat[-1]], X_raw[2, cat[0]] = -1.0, float(cards[cat[-1]]), np.nan
    params = synth.make_params(cfg, 500 + k)
    path = str(tmp_path / "m.tnw")
    synth.write_weights(params, path)
    _say(f"case random embedding {k} {prec}: {cfg} columns={cards.size} widest={dims.max()} B={B}")
    X = oe.embed(X_raw, cards, dims, tables).astype(np.float32)
    with tb.Model(path, prec) as m:
        m.set_embeddings(cards, dims, tables)
        lo_r, ag_r, ms_r = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
        lo, ag, ms = to_np(*m.forward(torch.from_numpy(X).cuda()))
    np.testing.assert_array_equal(lo_r, lo)
    np.testing.assert_allclose(ag_r, oe.reduce_columns(ag, dims), rtol=0, atol=2e-6)
    np.testing.assert_allclose(ms_r, oe.reduce_columns(ms, dims), rtol=0, atol=2e-6)
    if prec == "fp32":
        rlo, rag, rms = oe.forward_raw(params, X_raw, cards, dims, tables)
        rel = (np.abs(lo_r - rlo).max(1) / np.maximum(np.abs(rlo).max(1), 1e-2)).max()
        mt = 1e-5 * int(dims.max()) * max(1.0, cfg.gamma ** (cfg.n_steps - 1) / 2)
        _say(k, "logit_rel", rel, "agg", np.abs(ag_r - rag).max(), "step", np.abs(ms_r - rms).max(), "gate", mt)
        assert rel <= 1e-4
        assert np.abs(ag_r - rag).max() <= mt and np.abs(ms_r - rms).max() <= mt


@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 2000)])
def test_raw_fp32_matches_oracle(name, B, tmp_path):
    _say(f"case raw fp32 vs oracle {name} B={B}")
    params, m = model(name, "fp32", tmp_path)
    X_raw, cards, dims, tables = raw_rows(name, B)
    with m:
        m.set_embeddings(cards, dims, tables)
        lo, ag, ms = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
    rlo, rag, rms = oe.forward_raw(params, X_raw, cards, dims, tables)
    rel = (np.abs(lo - rlo).max(1) / np.maximum(np.abs(rlo).max(1), 1e-2)).max()
    cfg = synth.WORKLOADS[name]["cfg"]
    lt, mt = (1e-5, 1e-6 * max(1.0, cfg.gamma ** (cfg.n_steps - 1) / 2)) if name == "hr35" else (1e-4, 16e-5)
    _say(name, "logit_rel", rel, "agg", np.abs(ag - rag).max(), "step", np.abs(ms - rms).max())
    assert rel <= lt
    assert np.abs(ag - rag).max() <= mt and np.abs(ms - rms).max() <= mt
    np.testing.assert_allclose(ms.sum(-1), 1.0, atol=1e-5)


def test_raw_bf16_matches_oracle(tmp_path):
    _say("case raw bf16 vs oracle adult108")
    params, m = model("adult108", "bf16", tmp_path)
    X_raw, cards, dims, tables = raw_rows("adult108", 3000)
    with m:
        m.set_embeddings(cards, dims, tables)
        lo, ag, ms = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
    rlo, rag, rms = oe.forward_raw(params, X_raw, cards, dims, tables)
    assert np.abs(lo - rlo).max() <= 2e-2
    assert (lo.argmax(1) == rlo.argmax(1)).mean() >= 0.999
    assert np.abs(ag - rag).sum(-1).max() <= 1e-2 and np.abs(ms - rms).sum(-1).max() <= 2e-2


def test_invalid_levels_embed_to_zero(tmp_path):
    _say("case raw invalid levels")
    params, m = model("adult108", "fp32", tmp_path)
    X_raw, cards, dims, tables = raw_rows("adult108", 64)
    cat_cols = np.nonzero(cards)[0]
    bad = [-1.0, 1e9, 2.5, np.nan, np.inf, -0.5, float(cards[cat_cols[0]])]
    for k, v in enumerate(bad):
        X_raw[k, cat_cols[k % len(cat_cols)]] = v
    X_raw[10, cat_cols[0]] = float(cards[cat_cols[0]] - 1)     # the last valid level
    with m:
        m.set_embeddings(cards, dims, tables)
        lo, ag, ms = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
    rlo, rag, rms = oe.forward_raw(params, X_raw, cards, dims, tables)
    assert np.isfinite(lo).all()
    rel = (np.abs(lo - rlo).max(1) / np.maximum(np.abs(rlo).max(1), 1e-2)).max()
    assert rel <= 1e-4 and np.abs(ms - rms).max() <= 16e-5


def test_optional_steps_empty_batch_and_row_independence(tmp_path):
    _say("case raw optional steps / B=0 / row independence")
    params, m = model("adult108", "bf16", tmp_path)
    X_raw, cards, dims, tables = raw_rows("adult108", 700)
    with m:
        m.set_embeddings(cards, dims, tables)
        Xd = torch.from_numpy(X_raw).cuda()
        lo, ag, ms = m.forward_raw(Xd)
        lo2, ag2, none = m.forward_raw(Xd, with_steps=False)
        assert none is None
        sub = m.forward_raw(Xd[123:456].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(lo, lo2) and torch.equal(ag, ag2)
        assert torch.equal(sub[0], lo[123:456]) and torch.equal(sub[1], ag[123:456])
        assert torch.equal(sub[2], ms[:, 123:456])
        empty = torch.zeros((0, 14), dtype=torch.float32, device="cuda")
        r = m.forward_raw(empty)
        torch.cuda.synchronize()
        assert r[0].shape == (0, 2)


def test_embedding_spec_errors_and_replacement(tmp_path):
    _say("case raw spec errors")
    params, m = model("hr35", "fp32", tmp_path)
    X_raw, cards, dims, tables = raw_rows("hr35", 100)
    with m:
        with pytest.raises(tb.TabNetError) as e:      # no embedding yet
            m.forward_raw_into(torch.zeros((4, 35), device="cuda"), torch.zeros((4, 2), device="cuda"),
                               torch.zeros((4, 35), device="cuda"))
        assert e.value.status == tb.E_INVALID
        for c, d in [(cards, dims[:-1]), (cards, np.where(np.arange(35) == 0, 2, dims)),
                     (np.where(np.arange(35) == 30, -1, cards), dims)]:
            n = min(len(c), len(d))
            with pytest.raises((tb.TabNetError, ValueError)):
                m.set_embeddings(c[:n] if len(c) != len(d) else c, d, tables)
        # widths that do not add up to D
        with pytest.raises(tb.TabNetError):
            m.set_embeddings(cards[:-1], dims[:-1], tables[:-int(cards[-1])])
        # an all-continuous spec is the plain forward, and a later spec replaces it
        X = synth.make_inputs("hr", 100, synth.DATA_SEED["hr35"])
        m.set_embeddings(np.zeros(35), np.ones(35), np.zeros(0))
        a = to_np(*m.forward_raw(torch.from_numpy(X).cuda()))
        b = to_np(*m.forward(torch.from_numpy(X).cuda()))
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)
        m.set_embeddings(cards, dims, tables)
        c = to_np(*m.forward_raw(torch.from_numpy(X_raw).cuda()))
        np.testing.assert_array_equal(c[0], b[0])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_all_continuous_wide_layout_is_plain_forward(prec, tmp_path):
    # 108 raw columns: seven column tiles of the per-column reduction
    _say(f"case raw all-continuous 108 columns {prec}")
    params, m = model("adult108", prec, tmp_path)
    X = synth.make_inputs("adult", 777, synth.DATA_SEED["adult108"])
    with m:
        m.set_embeddings(np.zeros(108), np.ones(108), np.zeros(0))
        a = to_np(*m.forward_raw(torch.from_numpy(X).cuda()))
        b = to_np(*m.forward(torch.from_numpy(X).cuda()))
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_generic_raw_rows_need_fp32_or_bf16(tmp_path):
    """A generic-shape model has raw-row kernels in FP32 and BF16 only: in INT8 (which has
    generic embedded-row kernels) tabnet_set_embeddings is refused."""
    cfg = synth.TabNetConfig(D=150, n_d=48, n_a=48, n_steps=2, n_shared=1, n_indep=1, n_out=2, gamma=1.3)
    path = str(tmp_path / "g.tnw")
    synth.write_weights(synth.make_params(cfg, 8), path)
    rng = np.random.default_rng(9)
    cards, dims, tables = random_spec(cfg.D, rng)
    with tb.Model(path, "int8") as m:
        with pytest.raises(tb.TabNetError) as ei:
            m.set_embeddings(cards, dims, tables)
        assert ei.value.status == tb.E_UNSUPPORTED
