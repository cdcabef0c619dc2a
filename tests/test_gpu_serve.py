"""GPU serving: continuous batching must not change any request's result.

Requests of random sizes (some larger than one launch, so they are split) are served
in a mix; each request's logits and masks must be bit-identical to a tabnet_forward of
that request alone, and a sample is checked against the FP64 oracle."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import tabnet as oracle  # noqa: E402
from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def models(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    d = tmp_path_factory.mktemp("serve")
    out = {}
    for name in ("adult108", "hr35", "wide200", "wide512"):
        p = synth.make_params(synth.WORKLOADS[name]["cfg"], synth.WEIGHT_SEED[name])
        path = str(d / f"{name}.tnw")
        synth.write_weights(p, path)
        out[name] = (p, path)
    return out


def alone(model, X):
    lo, ag, ms = model.forward(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    return lo.cpu().numpy(), ag.cpu().numpy(), ms.cpu().numpy()


@pytest.mark.parametrize("use_graph", [True, False])
def test_mix_equals_alone(models, use_graph):
    pa, path_a = models["adult108"]
    ph, path_h = models["hr35"]
    _say(f"case serve mix use_graph={use_graph}")
    with tb.Model(path_a, "bf16") as ma, tb.Model(path_h, "bf16") as mh:
        cfgs = [ma.config, mh.config]
        rng = np.random.default_rng(7)
        Xa = synth.make_inputs("adult", 20000, 77)
        Xh = synth.make_inputs("hr", 5000, 78)
        reqs = []
        with tb.Server([ma, mh], max_rows_per_launch=2048, slots=3, with_step_masks=True,
                       use_graph=use_graph) as s:
            for k in range(120):
                m = 0 if k % 3 else 1
                pool = Xa if m == 0 else Xh
                rows = int(min(np.floor(np.exp(rng.uniform(0, np.log(4097)))), 4096))
                off = int(rng.integers(0, pool.shape[0] - rows))
                X = np.ascontiguousarray(pool[off:off + rows])
                c = cfgs[m]
                lo = np.full((rows, c.n_out), np.nan, np.float32)
                ag = np.full((rows, c.D), np.nan, np.float32)
                ms = np.full((c.n_steps, rows, c.D), np.nan, np.float32)
                reqs.append((m, X, lo, ag, ms, s.submit(m, X, lo, ag, ms)))
            for r in reqs:
                assert s.wait(r[5]) == tb.OK
            st = s.stats()
            _say("serve stats", {k: st[k] for k in ("completed", "launches", "mean_rows_per_launch", "p50_us", "p99_us")})
            assert st["completed"] == len(reqs)
        for m, X, lo, ag, ms, _ in reqs:
            a_lo, a_ag, a_ms = alone(ma if m == 0 else mh, X)
            np.testing.assert_array_equal(lo, a_lo)
            np.testing.assert_array_equal(ag, a_ag)
            np.testing.assert_array_equal(ms, a_ms)
        # a sample against the FP64 oracle (BF16 tolerances)
        for m, X, lo, ag, ms, _ in reqs[:6]:
            p = pa if m == 0 else ph
            rlo, rag, rms = oracle.forward(p, X[:64])
            assert np.abs(lo[:64] - rlo).max() <= 2e-2
            assert np.abs(ag[:64] - rag).sum(-1).max() <= 1e-2


@pytest.mark.parametrize("prec_a,prec_h", [("int8", "mxfp4"), ("mxfp8", "int8"), ("mxfp8_e5m2", "mxfp6_e3m2")])
def test_mix_quantised_equals_alone(models, prec_a, prec_h):
    """Quantised models (INT8, MX) served together: each request's outputs are those of the
    model's own forward of that request alone, bit for bit (the row coding is per row)."""
    _, path_a = models["adult108"]
    _, path_h = models["hr35"]
    _say(f"case serve quantised mix {prec_a} + {prec_h}")
    with tb.Model(path_a, prec_a) as ma, tb.Model(path_h, prec_h) as mh:
        cfgs = [ma.config, mh.config]
        rng = np.random.default_rng(11)
        pools = [synth.make_inputs("adult", 8000, 81), synth.make_inputs("hr", 3000, 82)]
        reqs = []
        with tb.Server([ma, mh], max_rows_per_launch=2048, slots=2, with_step_masks=True, use_graph=True) as s:
            for k in range(40):
                m = k % 2
                rows = int(min(np.floor(np.exp(rng.uniform(0, np.log(3001)))), 3000))
                off = int(rng.integers(0, pools[m].shape[0] - rows))
                X = np.ascontiguousarray(pools[m][off:off + rows])
                c = cfgs[m]
                lo = np.full((rows, c.n_out), np.nan, np.float32)
                ag = np.full((rows, c.D), np.nan, np.float32)
                ms = np.full((c.n_steps, rows, c.D), np.nan, np.float32)
                reqs.append((m, X, lo, ag, ms, s.submit(m, X, lo, ag, ms)))
            for r in reqs:
                assert s.wait(r[5]) == tb.OK
        for m, X, lo, ag, ms, _ in reqs:
            a_lo, a_ag, a_ms = alone(ma if m == 0 else mh, X)
            np.testing.assert_array_equal(lo, a_lo)
            np.testing.assert_array_equal(ag, a_ag)
            np.testing.assert_array_equal(ms, a_ms)


def test_serve_without_step_masks_and_tiny_requests(models):
    _, path_a = models["adult108"]
    _say("case serve tiny requests")
    with tb.Model(path_a, "fp32") as ma:
        X = synth.make_inputs("adult", 300, 5)
        with tb.Server([ma], max_rows_per_launch=64, slots=2) as s:
            outs = []
            for r in range(0, 300, 3):
                x = np.ascontiguousarray(X[r:r + 3])
                lo = np.empty((3, 2), np.float32)
                ag = np.empty((3, 108), np.float32)
                outs.append((r, lo, ag, s.submit(0, x, lo, ag)))
            for r, lo, ag, i in outs:
                assert s.wait(i) == tb.OK
        a_lo, a_ag, _ = alone(ma, X)
        for r, lo, ag, _ in outs:
            np.testing.assert_array_equal(lo, a_lo[r:r + 3])
            np.testing.assert_array_equal(ag, a_ag[r:r + 3])


def test_four_resident_models_mixed_equals_alone(models):
    """The multi-model load: four resident BF16 models (35, 108, 200 and 512 features; the
    last on the split-feature kernel) served together, the model drawn per request,
    1-8,192 rows per request (some split across launches).  Every request's logits and
    masks equal that model's own forward of the request alone, bit for bit, and a sample
    of rows of each model meets the BF16 gates against the FP64 oracle."""
    names = ["hr35", "adult108", "wide200", "wide512"]
    kinds = {"hr35": "hr", "adult108": "adult", "wide200": "wide", "wide512": "wide512"}
    _say("case serve four models bf16")
    ms_ = [tb.Model(models[n][1], "bf16") for n in names]
    try:
        cfgs = [m.config for m in ms_]
        pools = [synth.make_inputs(kinds[n], 12000, 90 + k) for k, n in enumerate(names)]
        rng = np.random.default_rng(23)
        reqs = []
        with tb.Server(ms_, max_rows_per_launch=8192, slots=3, with_step_masks=True, use_graph=True) as s:
            for k in range(48):
                m = int(rng.integers(0, 4))
                rows = int(min(np.floor(np.exp(rng.uniform(0, np.log(8193)))), 8192))
                off = int(rng.integers(0, pools[m].shape[0] - rows + 1))
                X = np.ascontiguousarray(pools[m][off:off + rows])
                c = cfgs[m]
                lo = np.full((rows, c.n_out), np.nan, np.float32)
                ag = np.full((rows, c.D), np.nan, np.float32)
                mk = np.full((c.n_steps, rows, c.D), np.nan, np.float32)
                reqs.append((m, X, lo, ag, mk, s.submit(m, X, lo, ag, mk)))
            for r in reqs:
                assert s.wait(r[5]) == tb.OK
            st = s.stats()
            _say("serve stats", {k: st[k] for k in ("completed", "launches", "mean_rows_per_launch", "p99_us")})
        assert sorted({r[0] for r in reqs}) == [0, 1, 2, 3]
        for m, X, lo, ag, mk, _ in reqs:
            a_lo, a_ag, a_ms = alone(ms_[m], X)
            np.testing.assert_array_equal(lo, a_lo)
            np.testing.assert_array_equal(ag, a_ag)
            np.testing.assert_array_equal(mk, a_ms)
        for m in range(4):
            m_reqs = [r for r in reqs if r[0] == m]
            X, lo, ag = m_reqs[0][1][:32], m_reqs[0][2][:32], m_reqs[0][3][:32]
            rlo, rag, _ = oracle.forward(models[names[m]][0], X)
            assert np.abs(lo - rlo).max() <= 2e-2
            assert np.abs(ag - rag).sum(-1).max() <= 1e-2
    finally:
        for m in ms_:
            m.close()


def test_generic_shape_models_served(tmp_path):
    """Models outside the exact shape families (generic kernels: D = 150 with n_d = n_a = 48
    in BF16, D = 300 with n_d = n_a = 40 on the split-feature kernel in INT8) served beside
    each other: every request equals a tabnet_forward of it alone, bit for bit."""
    cfgs = [synth.TabNetConfig(D=150, n_d=48, n_a=48, n_steps=4, n_shared=2, n_indep=2, n_out=2, gamma=1.3),
            synth.TabNetConfig(D=300, n_d=40, n_a=40, n_steps=5, n_shared=2, n_indep=1, n_out=3, gamma=1.5)]
    paths = []
    for i, c in enumerate(cfgs):
        paths.append(str(tmp_path / f"g{i}.tnw"))
        synth.write_weights(synth.make_params(c, 4400 + i), paths[-1])
    _say("case serve generic-shape models")
    with tb.Model(paths[0], "bf16") as m0, tb.Model(paths[1], "int8") as m1:
        ms_ = [m0, m1]
        rng = np.random.default_rng(11)
        pools = [synth.make_normal_inputs(3000, c.D, 4500 + i) for i, c in enumerate(cfgs)]
        reqs = []
        with tb.Server(ms_, max_rows_per_launch=1024, slots=3, with_step_masks=True) as s:
            for k in range(40):
                m = k % 2
                c = cfgs[m]
                rows = int(rng.integers(1, 2000))
                off = int(rng.integers(0, pools[m].shape[0] - rows))
                X = np.ascontiguousarray(pools[m][off:off + rows])
                lo = np.full((rows, c.n_out), np.nan, np.float32)
                ag = np.full((rows, c.D), np.nan, np.float32)
                mk = np.full((c.n_steps, rows, c.D), np.nan, np.float32)
                reqs.append((m, X, lo, ag, mk, s.submit(m, X, lo, ag, mk)))
            for r in reqs:
                assert s.wait(r[5]) == tb.OK
        for m, X, lo, ag, mk, _ in reqs:
            a_lo, a_ag, a_ms = alone(ms_[m], X)
            np.testing.assert_array_equal(lo, a_lo)
            np.testing.assert_array_equal(ag, a_ag)
            np.testing.assert_array_equal(mk, a_ms)
