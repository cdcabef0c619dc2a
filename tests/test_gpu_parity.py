"""GPU parity: libtabnet (HIP, gfx950) against the FP64 oracle on seeded inputs.

Tolerances (logits per row, masks per entry or per row):
  FP32: logits |d| <= 1e-5 max(|ref|_inf, 1e-2), masks |d| <= 1e-6 max(1, gamma^(S-1) / 2)
  (an FP32 score |z| of size 2^k carries a rounding unit of 2^(k-24), and the prior can
  grow scores to gamma^(S-1)).
  BF16 against FP64: logits |d| <= 2e-2, per-row L1 of the aggregate mask <= 1e-2,
  argmax agreement >= 99.9 %, per-row L1 of each step mask <= 2e-2 (an FP64 forward on
  the same bf16-rounded operands already reaches 1.6e-2 on the worst Adult-shaped row of
  these batches and 2.0e-2 over the full batch, so 1e-2 is beyond the format).  BF16
  against FP64 on bf16-rounded operands (the oracle's rounding option) isolates the
  kernel: logits |d| <= 1e-3, mask L1 <= 5e-3.
Every row of the benchmarked launches is compared in test_gpu_fullsize.py.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import tabnet as oracle  # noqa: E402
from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402
from paper_2510_19689_amd.synth import TabNetConfig  # noqa: E402

pytestmark = pytest.mark.gpu

MX_FORMATS = ["mxfp8", "mxfp8_e5m2", "mxfp6", "mxfp6_e3m2", "mxfp4"]


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    if not os.path.exists(tb.LIB_PATH):
        pytest.fail("libtabnet.so not built")
    return torch.device("cuda", 0)


def load(params, tmp_path, prec, name="m"):
    path = str(tmp_path / f"{name}.tnw")
    synth.write_weights(params, path)
    return tb.Model(path, prec)


def run(model, X, with_steps=True):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    lo, ag, ms = model.outputs(X.shape[0], with_steps)
    for t in (lo, ag, ms):
        if t is not None:
            t.fill_(float("nan"))
    model.forward_into(Xd, lo, ag, ms)
    torch.cuda.synchronize()
    return lo.cpu().numpy(), ag.cpu().numpy(), None if ms is None else ms.cpu().numpy()


def errs(got, ref):
    (lo, ag, ms), (rlo, rag, rms) = got, ref
    return dict(
        logit_abs=float(np.abs(lo - rlo).max()),
        logit_rel=float((np.abs(lo - rlo).max(1) / np.maximum(np.abs(rlo).max(1), 1e-2)).max()),
        agg_abs=float(np.abs(ag - rag).max()),
        step_abs=float(np.abs(ms - rms).max()) if ms is not None else 0.0,
        agg_l1=float(np.abs(ag - rag).sum(-1).max()),
        step_l1=float(np.abs(ms - rms).sum(-1).max()) if ms is not None else 0.0,
        argmax=float((lo.argmax(1) == rlo.argmax(1)).mean()))


def check_fp32_tight(got, ref, tag, cfg=None):
    e = errs(got, ref)
    _say(tag, e)
    assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
    assert e["logit_rel"] <= 1e-5, e
    mtol = 1e-6 if cfg is None else 1e-6 * max(1.0, cfg.gamma ** (cfg.n_steps - 1) / 2)
    assert e["agg_abs"] <= mtol and e["step_abs"] <= mtol, e


@pytest.mark.parametrize("B", [1, 7, 63, 64, 65, 129, 256, 1000])
def test_fp32_hr35(tmp_path, B):
    params = synth.make_params(synth.WORKLOADS["hr35"]["cfg"], synth.WEIGHT_SEED["hr35"])
    X = synth.make_inputs("hr", B, synth.DATA_SEED["hr35"])
    _say(f"case fp32 hr35 B={B}")
    with load(params, tmp_path, "fp32") as m:
        got = run(m, X)
    check_fp32_tight(got, oracle.forward(params, X), f"fp32 hr35 B={B}")


SMALL = [
    dict(D=7, n_d=3, n_a=2, n_steps=3, n_shared=2, n_indep=2, n_out=2, gamma=1.3),
    dict(D=20, n_d=5, n_a=6, n_steps=4, n_shared=1, n_indep=1, n_out=3, gamma=1.5),
    dict(D=33, n_d=8, n_a=8, n_steps=2, n_shared=0, n_indep=3, n_out=1, gamma=1.2),
    dict(D=48, n_d=4, n_a=12, n_steps=5, n_shared=3, n_indep=0, n_out=5, gamma=2.0),
    dict(D=64, n_d=16, n_a=16, n_steps=3, n_shared=2, n_indep=2, n_out=4, gamma=1.3),
    dict(D=1, n_d=1, n_a=1, n_steps=2, n_shared=1, n_indep=1, n_out=1, gamma=1.0),
]


@pytest.mark.parametrize("k", range(len(SMALL)))
def test_fp32_small_shapes(tmp_path, k):
    cfg = TabNetConfig(**SMALL[k])
    params = synth.make_params(cfg, 100 + k)
    X = synth.make_normal_inputs(300, cfg.D, seed=200 + k)
    _say(f"case fp32 small {SMALL[k]}")
    with load(params, tmp_path, "fp32") as m:
        got = run(m, X)
    check_fp32_tight(got, oracle.forward(params, X), f"fp32 small {k}", cfg)


@pytest.mark.parametrize("name,B", [("adult108", 2000), ("wide200", 300)])
def test_fp32_wide_models(tmp_path, name, B):
    params, X = synth.workload(name, rows=B)
    _say(f"case fp32 {name} B={B}")
    with load(params, tmp_path, "fp32") as m:
        got = run(m, X)
    check_fp32_tight(got, oracle.forward(params, X), f"fp32 {name}", params["config"])


def check_reduced(got, params, X, weights, acts, tag, tol=(1e-3, 5e-3, 5e-3)):
    """Against FP64 on the same rounded operands (logit |d|, aggregate and step mask L1 per
    row <= tol); returns the errors against plain FP64 for the caller's own gates."""
    ref = oracle.forward(params, X)
    e = errs(got, ref)
    _say(tag, "vs fp64", e)
    emu = oracle.forward(params, X, weights=weights, acts=acts)
    e2 = errs(got, emu)
    _say(tag, "vs rounded-operand fp64", e2)
    assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
    assert e2["logit_abs"] <= tol[0] and e2["agg_l1"] <= tol[1] and e2["step_l1"] <= tol[2], e2
    return e


@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 3000), ("wide200", 400)])
def test_bf16_parity(tmp_path, name, B):
    params, X = synth.workload(name, rows=B)
    _say(f"case bf16 {name} B={B}")
    with load(params, tmp_path, "bf16") as m:
        got = run(m, X)
    e = check_reduced(got, params, X, "bf16", "bf16", f"bf16 {name}")
    assert e["logit_abs"] <= 2e-2, e
    assert e["argmax"] >= 0.999, e
    assert e["agg_l1"] <= 1e-2 and e["step_l1"] <= 2e-2, e


@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 3000), ("wide200", 400)])
def test_fp8_weights_parity(tmp_path, name, B):
    """E4M3 weights (one scale per output channel) with BF16 GEMM inputs: against FP64 on
    the same operands (E4M3 weights, bf16-rounded inputs) with the BF16 kernel gates, and
    against plain FP64 with the logit and argmax gates of the target."""
    params, X = synth.workload(name, rows=B)
    _say(f"case fp8 weights {name} B={B}")
    with load(params, tmp_path, "fp8w") as m:
        got = run(m, X)
    e = check_reduced(got, params, X, "e4m3", "bf16", f"fp8w {name}", tol=(2e-3, 1.5e-2, 2e-2))
    assert e["logit_abs"] <= 2e-2 and e["argmax"] >= 0.999, e


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp8w", "int8"] + MX_FORMATS)
def test_optional_step_masks_and_empty_batch(tmp_path, prec):
    params, X = synth.workload("adult108", rows=777)
    _say(f"case masks_step NULL {prec}")
    with load(params, tmp_path, prec) as m:
        a = run(m, X, with_steps=True)
        b = run(m, X, with_steps=False)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        lo, ag, ms = m.outputs(0)
        m.forward_into(torch.empty((0, 108), device="cuda"), lo, ag, ms)
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8w", "int8"])
def test_rows_independent_and_deterministic(tmp_path, prec):
    """A row's outputs are bit-identical whatever batch it is in and on every run."""
    params, X = synth.workload("adult108", rows=1000)
    _say(f"case row independence {prec}")
    with load(params, tmp_path, prec) as m:
        full = run(m, X)
        again = run(m, X)
        for u, v in zip(full, again):
            np.testing.assert_array_equal(u, v)
        for lo_, hi_ in ((0, 1), (5, 6), (999, 1000), (17, 83), (500, 1000)):
            part = run(m, X[lo_:hi_])
            np.testing.assert_array_equal(part[0], full[0][lo_:hi_])
            np.testing.assert_array_equal(part[1], full[1][lo_:hi_])
            np.testing.assert_array_equal(part[2], full[2][:, lo_:hi_])


@pytest.mark.parametrize("prec", ["bf16", "fp8", "fp8w", "int8"] + MX_FORMATS)
def test_nonfinite_row_is_contained(tmp_path, prec):
    """A NaN or Inf in a row changes nothing in the other rows; in the scaled formats the
    row (or block) scale is taken from that row alone."""
    params, X = synth.workload("hr35", rows=200)
    Xb = X.copy()
    Xb[3, 5] = np.nan
    Xb[150, :] = np.inf
    Xb[77, 2] = -np.inf
    _say(f"case non-finite rows {prec}")
    with load(params, tmp_path, prec) as m:
        clean = run(m, X)
        dirty = run(m, Xb)
    keep = np.ones(200, bool)
    keep[[3, 77, 150]] = False
    for u, v in zip(clean, dirty):
        if u.ndim == 3:
            np.testing.assert_array_equal(u[:, keep], v[:, keep])
        else:
            np.testing.assert_array_equal(u[keep], v[keep])


def run_full_sampled(m, X, idx):
    """One launch over every row of X with step masks on (the launch the benchmark times);
    the invariants are checked on the device for every row (finite, non-negative, each
    step mask sums to 1, each aggregate mask sums to 1 or is a zero row), and only the
    rows idx come back to the host."""
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    lo, ag, ms = m.outputs(X.shape[0], True)
    for t in (lo, ag, ms):
        t.fill_(float("nan"))
    m.forward_into(Xd, lo, ag, ms)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(lo).all()) and bool(torch.isfinite(ag).all()) and bool(torch.isfinite(ms).all())
    assert bool((ms >= 0).all()) and bool((ag >= 0).all())
    assert float((ms.sum(-1) - 1).abs().max()) <= 2e-5
    sa = ag.sum(-1)
    assert bool((((sa - 1).abs() <= 2e-5) | (sa == 0)).all())
    it = torch.from_numpy(idx).cuda()
    out = lo[it].cpu().numpy(), ag[it].cpu().numpy(), ms[:, it].cpu().numpy()
    del Xd, lo, ag, ms, sa
    return out


@pytest.fixture(scope="module")
def wide200_full():
    """The 200-feature workload at its full batch (1,048,576 rows), 384 sampled rows (the
    first, the last, the middle and 381 at random) and plain FP64 on those rows."""
    params, X = synth.workload("wide200")
    assert X.shape == (1048576, 200)
    n = X.shape[0]
    idx = np.random.default_rng(0).choice(n, 384, replace=False)
    idx[:3] = [0, n - 1, n // 2]
    return params, X, idx, oracle.forward(params, X[idx])


@pytest.mark.parametrize("prec", ["int8"] + MX_FORMATS)
def test_full_size_wide200_sampled(tmp_path, wide200_full, prec):
    """The 200-feature model at its full batch (1,048,576 rows, 7 steps, step masks on), in
    the launch configuration of `bench.py --workload wide200`, in the formats that are not
    compared on every row (FP32, BF16 and FP8 are, in test_gpu_fullsize.py): invariants on
    every row, sampled rows against the oracle with the gates of the smaller cases.  On
    these rows the formats themselves move (logits, aggregate L1, step L1) by at most
    (2.2e-3, 8.8e-3, 2.8e-2) in INT8 and (2.9e-2, 0.16, 0.56) in MXFP4, the largest among
    the MX formats."""
    params, X, idx, ref = wide200_full
    _say(f"case full wide200 {prec}")
    with load(params, tmp_path, prec) as m:
        got = run_full_sampled(m, X, idx)
    e = errs(got, ref)
    _say(f"full wide200 {prec} sampled", e)
    oracle_fmt, worst, typical = ROW_GATES[prec]
    check_rows_on_rounded(got, params, X[idx], oracle_fmt, f"full wide200 {prec}", worst=worst, typical=typical)
    lo_t, agg_t, step_t = FP64_GATES[prec]
    assert e["logit_abs"] <= lo_t and e["agg_l1"] <= agg_t and e["step_l1"] <= step_t, e
    assert e["argmax"] >= 0.995, e


@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 3000), ("wide200", 400)])
def test_fp8_parity(tmp_path, name, B):
    """E4M3 weights (one scale per output channel) and E4M3 GEMM inputs (one scale per row,
    max |u| / 448), FP32 sums on the FP8 matrix cores.

    Row by row against FP64 on the same E4M3 operands (check_rows_on_rounded); the FP8
    instruction's sums, like the scaled one's, need not be exact FP32 sums, so the typical
    row is gated at the median within 1e-4.  Against plain FP64 the format decides: the
    oracle on E4M3 operands differs from plain FP64 by up to (logits, aggregate L1, step L1)
    = (1.3e-2, 9.2e-2, 0.18) on these rows with argmax unchanged; the gates leave more."""
    params, X = synth.workload(name, rows=B)
    _say(f"case fp8 {name} B={B}")
    with load(params, tmp_path, "fp8") as m:
        got = run(m, X)
    check_rows_on_rounded(got, params, X, "e4m3", f"fp8 {name}", worst=(0.1, 0.05, 5e-3), typical=(0.5, 1e-4))
    e = errs(got, oracle.forward(params, X))
    _say(f"fp8 {name} vs fp64", e)
    lo_t, agg_t, step_t = FP64_GATES["fp8"]
    assert e["logit_abs"] <= lo_t and e["agg_l1"] <= agg_t and e["step_l1"] <= step_t, e
    assert e["argmax"] >= 0.999, e


def check_int8(got, params, X, tag):
    check_rows_on_rounded(got, params, X, "int8", tag, worst=(2.5e-2, 1e-2, 2e-3))


def check_rows_on_rounded(got, params, X, fmt, tag, worst, typical=(0.9, 1e-5)):
    """A quantised path against FP64 on the same quantised operands, row by row.

    The kernel forms its GEMM inputs in FP32; where such an input lands on the other side
    of a rounding boundary than its FP64 value, its code moves by one, which moves that
    GEMM's outputs by sigma_n * step * |Wq_nk|: one element's share of the format's own
    rounding error, carried through the later layers and the sparsemax.  An FP32/FP64
    difference of ~1e-7 of a step makes such flips rare, so most rows agree to FP32
    rounding and a few rows move by a fraction of what INT8 itself moves them from FP64.
    Gates: a share `typical` = (fraction, bound) of rows within the bound (step-mask L1 and
    logits), by default 90 % within 1e-5; every row within `worst` = (step L1, aggregate
    L1, logits), for INT8 2.5e-2, 1e-2 and 2e-3.  A wrong index, scale or code in the
    kernel moves every row by far more, not a few rows.  (MX formats: a flip is rarer,
    since the FP32/FP64 difference must cross an element boundary of a grid 2^-3 (E4M3)
    or 2^-1 (E2M1) wide relative to the value, but larger.)"""
    lo, ag, ms = got
    rlo, rag, rms = oracle.forward(params, X, weights=fmt, acts=fmt)
    step = np.abs(ms - rms).sum(-1).max(0)
    agg = np.abs(ag - rag).sum(-1)
    logit = np.abs(lo - rlo).max(1)
    q = lambda v: [float(np.percentile(v, p)) for p in (50, 90, 99, 100)]
    _say(tag, f"vs {fmt}-operand fp64 per row p50/p90/p99/max: step L1", q(step), "agg L1", q(agg), "logits", q(logit),
         "rows moved:", float((step > 1e-5).mean()))
    assert np.isfinite(lo).all() and np.isfinite(ag).all()
    frac, bound = typical
    assert (step <= bound).mean() >= frac and (logit <= bound).mean() >= frac
    assert step.max() <= worst[0] and agg.max() <= worst[1] and logit.max() <= worst[2]


@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 3000), ("wide200", 400)])
def test_int8_parity(tmp_path, name, B):
    """INT8 weights (one scale per output channel) and INT8 GEMM inputs (one step per row),
    exact INT32 products: row by row against FP64 on the same operands (check_int8), and
    against plain FP64 with the gates of the E4M3-weight path (the format decides there)."""
    params, X = synth.workload(name, rows=B)
    _say(f"case int8 {name} B={B}")
    with load(params, tmp_path, "int8") as m:
        got = run(m, X)
    check_int8(got, params, X, f"int8 {name}")
    e = errs(got, oracle.forward(params, X))
    _say(f"int8 {name} vs fp64", e)
    lo_t, agg_t, step_t = FP64_GATES["int8"]
    assert e["logit_abs"] <= lo_t and e["agg_l1"] <= agg_t and e["step_l1"] <= step_t, e
    assert e["argmax"] >= 0.995, e


def test_int8_wide_loads_and_round_trip(tmp_path):
    """The 512-feature model loads in INT8 (split-feature kernel), and a handle reports
    its precision."""
    cfg = synth.WORKLOADS["wide512"]["cfg"]
    params = synth.make_params(cfg, 3)
    path = str(tmp_path / "w.tnw")
    synth.write_weights(params, path)
    with tb.Model(path, "int8") as m:
        assert tb.lib().tabnet_get_precision(m._h) == tb.INT8
    params, X = synth.workload("hr35", rows=40)
    with load(params, tmp_path, "int8") as m:
        assert tb.lib().tabnet_get_precision(m._h) == tb.INT8


# Against plain FP64 the MX formats' own error decides: the oracle on MX operands differs
# from plain FP64 by up to (logits, aggregate L1, step L1) = (1.2e-2, 0.22, 0.31) in MXFP8
# and (3.3e-2, 0.45, 0.86) in MXFP4 on these rows (MXFP6 below), with argmax unchanged; the gates leave
# a quarter more.  Per row against the same MX operands: flips of an E2M1 element move a
# value by up to a third, hence the wider worst-row bounds for MXFP4.  The E4M3 form of
# the scaled MFMA does not sum its products exactly in FP32: on known operands it
# differs from the exact dot product by up to 5.2e-6 of sum |a_k b_k| (the E2M1 form is
# exact), so every MXFP8 GEMM output carries an error of that order and the typical
# MXFP8 row moves by ~1e-5; its typical-row gate is the median row within 1e-4.
MX_GATES = {"mxfp8": dict(fp64=(1.5e-2, 0.28, 0.4), worst=(0.1, 0.05, 5e-3), typical=(0.5, 1e-4)),
            # MXFP6 (E2M3): format error (1.3e-2, 0.097, 0.27); its instruction form sums exactly
            "mxfp6": dict(fp64=(1.7e-2, 0.125, 0.35), worst=(0.1, 0.05, 5e-3), typical=(0.9, 1e-5)),
            "mxfp4": dict(fp64=(4.2e-2, 0.56, 1.08), worst=(0.4, 0.2, 2e-2), typical=(0.9, 1e-5)),
            # E5M2 and E3M2 elements carry two mantissa bits (a flip moves a value by up to an
            # eighth): format error (1.8e-2, 0.19, 0.39) and (2.0e-2, 0.20, 0.41).  The 8-bit form
            # of the instruction sums as the E4M3 one does; the 6-bit form as E2M3.
            "mxfp8_e5m2": dict(fp64=(2.3e-2, 0.24, 0.49), worst=(0.2, 0.1, 1e-2), typical=(0.5, 1e-4)),
            "mxfp6_e3m2": dict(fp64=(2.5e-2, 0.25, 0.51), worst=(0.2, 0.1, 1e-2), typical=(0.9, 1e-5))}


@pytest.mark.parametrize("fmt", MX_FORMATS)
@pytest.mark.parametrize("name,B", [("hr35", 256), ("adult108", 3000), ("wide200", 400)])
def test_mx_parity(tmp_path, name, B, fmt):
    """OCP MX formats on both GEMM operands (E8M0 block scales applied by the scaled MFMA)."""
    params, X = synth.workload(name, rows=B)
    _say(f"case {fmt} {name} B={B}")
    with load(params, tmp_path, fmt) as m:
        got = run(m, X)
    gates = MX_GATES[fmt]
    check_rows_on_rounded(got, params, X, fmt, f"{fmt} {name}", worst=gates["worst"], typical=gates["typical"])
    e = errs(got, oracle.forward(params, X))
    _say(f"{fmt} {name} vs fp64", e)
    lo_t, agg_t, step_t = gates["fp64"]
    assert e["logit_abs"] <= lo_t and e["agg_l1"] <= agg_t and e["step_l1"] <= step_t, e
    assert e["argmax"] >= 0.995, e
    lo, ag, ms = got
    np.testing.assert_allclose(ms.sum(-1), 1.0, atol=2e-5)
    np.testing.assert_allclose(ag.sum(-1), 1.0, atol=2e-5)


@pytest.mark.parametrize("fmt", MX_FORMATS)
def test_mx_rows_independent_and_wide_loads(tmp_path, fmt):
    """A row's outputs do not depend on its sub-batch; the 512-feature model loads in every
    MX form (split-feature kernel)."""
    params, X = synth.workload("adult108", rows=300)
    _say(f"case {fmt} row independence")
    with load(params, tmp_path, fmt) as m:
        full = run(m, X)
        for lo_, hi_ in ((0, 1), (17, 83), (299, 300)):
            part = run(m, X[lo_:hi_])
            for u, v in zip(part[:2], full[:2]):
                np.testing.assert_array_equal(u, v[lo_:hi_])
            np.testing.assert_array_equal(part[2], full[2][:, lo_:hi_])
    cfg = synth.WORKLOADS["wide512"]["cfg"]
    path = str(tmp_path / "w.tnw")
    synth.write_weights(synth.make_params(cfg, 3), path)
    with tb.Model(path, fmt) as m:
        assert m.config.D == 512


# per-row gates of each scaled format against FP64 on its own operands (see the tests above)
# Against plain FP64: (logits, aggregate L1, step L1) per scaled format.
FP64_GATES = {"fp8": (2e-2, 0.12, 0.25), "int8": (5e-2, 0.1, 0.25),
              **{f: MX_GATES[f]["fp64"] for f in MX_FORMATS}}

ROW_GATES = {"int8": ("int8", (2.5e-2, 1e-2, 2e-3), (0.9, 1e-5)),
             "fp8": ("e4m3", (0.1, 0.05, 5e-3), (0.5, 1e-4)),
             **{f: (f, MX_GATES[f]["worst"], MX_GATES[f]["typical"]) for f in MX_FORMATS}}


# Compiled register-resident shape families: (D range, n_d + n_a range, n_d range), i.e.
# 16-feature tiles DT = 1, 2, 3, 4 with one hidden tile, DT = 4 with two, 7 with four and 13
# with eight (and the matching first attention tile).
FAMILIES = [((1, 16), (2, 16), (1, 15)), ((17, 32), (2, 16), (1, 15)), ((33, 48), (2, 16), (1, 15)),
            ((49, 64), (2, 16), (1, 15)), ((49, 64), (17, 32), (16, 31)), ((97, 112), (49, 64), (32, 47)),
            ((193, 208), (113, 128), (64, 79))]


def random_config(k):
    """Seeded model configuration k: family k mod 7, widths, 1-6 steps, 0-3 shared and 0-3
    step layers (at least one), 1-8 outputs, gamma in [1, 2), and a batch of 1-259 rows."""
    rng = np.random.default_rng(5000 + k)
    (d0, d1), (N0, N1), (nd0, nd1) = FAMILIES[k % len(FAMILIES)]
    D = int(rng.integers(d0, d1 + 1))
    n_d = int(rng.integers(nd0, nd1 + 1))
    N = int(rng.integers(max(N0, n_d + 1), N1 + 1))
    n_sh, n_ind = int(rng.integers(0, 4)), int(rng.integers(0, 4))
    if n_sh + n_ind == 0:
        n_ind = 1
    cfg = TabNetConfig(D=D, n_d=n_d, n_a=N - n_d, n_steps=int(rng.integers(1, 7)), n_shared=n_sh, n_indep=n_ind,
                       n_out=int(rng.integers(1, 9)), gamma=float(rng.uniform(1.0, 2.0)))
    return cfg, int(rng.integers(1, 260))


@pytest.mark.parametrize("k", range(14))
def test_random_configurations(tmp_path, k):
    """Two seeded random models per compiled shape family: FP32 against FP64 with the gates
    of the small models (check_fp32_tight: logits 1e-5 relative, masks 1e-6 times the
    prior's growth max(1, gamma^(S-1) / 2); measured at most 4.4e-6 and 1.0e-6), BF16 against FP64
    on bf16-rounded operands (check_reduced), and one scaled format (in turn) against FP64
    on its own operands with its row gates."""
    cfg, B = random_config(k)
    fmt = list(ROW_GATES)[k % len(ROW_GATES)]
    params = synth.make_params(cfg, 6000 + k)
    X = synth.make_normal_inputs(B, cfg.D, seed=7000 + k)
    _say(f"case random configuration {k}: {cfg} B={B}, scaled format {fmt}")
    ref = oracle.forward(params, X)
    with load(params, tmp_path, "fp32", "a") as m:
        check_fp32_tight(run(m, X), ref, f"random {k} fp32", cfg)
    with load(params, tmp_path, "bf16", "b") as m:
        check_reduced(run(m, X), params, X, "bf16", "bf16", f"random {k} bf16")
    if fmt in MX_FORMATS and cfg.n_d % 16 and cfg.n_d % 16 + cfg.n_a > 32:
        # the attention half's MX blocks would straddle the kernel's tile pairs: refused,
        # and the row-coded FP8 path is checked on this model instead
        with pytest.raises(tb.TabNetError) as ei:
            load(params, tmp_path, fmt, "c")
        assert ei.value.status == tb.E_UNSUPPORTED
        fmt = "fp8"
    oracle_fmt, worst, typical = ROW_GATES[fmt]
    with load(params, tmp_path, fmt, "c") as m:
        got = run(m, X)
    check_rows_on_rounded(got, params, X, oracle_fmt, f"random {k} {fmt}", worst=worst,
                          typical=typical if B >= 50 else (0.0, 1.0))


@pytest.mark.parametrize("fmt", list(ROW_GATES))
@pytest.mark.parametrize("k", range(len(SMALL)))
def test_scaled_formats_small_shapes(tmp_path, k, fmt):
    """The scaled formats on the small shapes: attention halves that start 1, 3, 4, 5 or 8
    channels into a tile (the row scales and MX blocks of the attentive GEMM cover the
    attention channels only, at their positions in h's tiles), no shared or no step
    layers, a single feature."""
    cfg = TabNetConfig(**SMALL[k])
    params = synth.make_params(cfg, 100 + k)
    X = synth.make_normal_inputs(300, cfg.D, seed=200 + k)
    _say(f"case {fmt} small shape {k}: {SMALL[k]}")
    oracle_fmt, worst, typical = ROW_GATES[fmt]
    with load(params, tmp_path, fmt) as m:
        got = run(m, X)
    check_rows_on_rounded(got, params, X, oracle_fmt, f"{fmt} small {k}", worst=worst, typical=typical)


# Models between the exact shape families, served by the generic kernels (FP32 and BF16,
# compiled for up to 16 DT features and 16 NT hidden channels, DT in {4, 8, 13}, NT in
# {1, 2, 4, 8}): named cases, then seeded random ones drawn outside FAMILIES.
GENERIC = [dict(D=150, n_d=48, n_a=48, n_steps=4, n_shared=2, n_indep=2, n_out=2, gamma=1.3),
           dict(D=100, n_d=20, n_a=20, n_steps=3, n_shared=1, n_indep=1, n_out=3, gamma=1.5),
           dict(D=50, n_d=24, n_a=24, n_steps=5, n_shared=2, n_indep=0, n_out=2, gamma=1.2),
           dict(D=20, n_d=8, n_a=40, n_steps=2, n_shared=0, n_indep=2, n_out=5, gamma=1.8),
           dict(D=180, n_d=70, n_a=50, n_steps=6, n_shared=0, n_indep=3, n_out=4, gamma=1.6)]


def in_family(cfg):
    return any(d0 <= cfg.D <= d1 and N0 <= cfg.N <= N1 and nd0 <= cfg.n_d <= nd1
               for (d0, d1), (N0, N1), (nd0, nd1) in FAMILIES)


def random_generic(k):
    """Seeded model k outside the exact families: D 1-208, n_d + n_a 2-128, 1-6 steps, 0-3
    shared and 0-3 step layers (at least one), 1-8 outputs, gamma in [1, 2); 1-259 rows."""
    rng = np.random.default_rng(5500 + k)
    while True:
        D = int(rng.integers(1, 209))
        N = int(rng.integers(2, 129))
        n_d = int(rng.integers(1, N))
        n_sh, n_ind = int(rng.integers(0, 4)), int(rng.integers(0, 4))
        if n_sh + n_ind == 0:
            n_ind = 1
        cfg = TabNetConfig(D=D, n_d=n_d, n_a=N - n_d, n_steps=int(rng.integers(1, 7)), n_shared=n_sh,
                           n_indep=n_ind, n_out=int(rng.integers(1, 9)), gamma=float(rng.uniform(1.0, 2.0)))
        B = int(rng.integers(1, 260))
        if not in_family(cfg):
            return cfg, B


@pytest.mark.parametrize("k", range(len(GENERIC) + 8))
def test_generic_shapes(tmp_path, k):
    """Models outside the exact shape families run on the generic kernels: FP32 against
    FP64 with the small models' gates (check_fp32_tight), BF16 against FP64 on bf16-rounded
    operands (check_reduced), FP8 weights against FP64 on E4M3 weights and bf16 inputs (the
    register kernel's FP8-weight gates), and FP8 on both operands and INT8 against FP64 on
    their coded operands (their row gates); a row's outputs do not depend on its sub-batch,
    and without step masks the logits and aggregate masks are unchanged bit for bit."""
    if k < len(GENERIC):
        cfg, B = TabNetConfig(**GENERIC[k]), 300
    else:
        cfg, B = random_generic(k)
    assert not in_family(cfg)
    params = synth.make_params(cfg, 8800 + k)
    X = synth.make_normal_inputs(B, cfg.D, seed=8900 + k)
    _say(f"case generic shape {k}: {cfg} B={B}")
    ref = oracle.forward(params, X)
    with load(params, tmp_path, "fp32", "a") as m:
        got = run(m, X)
        check_fp32_tight(got, ref, f"generic {k} fp32", cfg)
        lo_, hi_ = B // 3, min(B, B // 3 + 17)
        part = run(m, X[lo_:hi_])
        np.testing.assert_array_equal(part[0], got[0][lo_:hi_])
        np.testing.assert_array_equal(part[1], got[1][lo_:hi_])
        np.testing.assert_array_equal(part[2], got[2][:, lo_:hi_])
        nomask = run(m, X, with_steps=False)
        np.testing.assert_array_equal(nomask[0], got[0])
        np.testing.assert_array_equal(nomask[1], got[1])
        assert nomask[2] is None
    with load(params, tmp_path, "bf16", "b") as m:
        check_reduced(run(m, X), params, X, "bf16", "bf16", f"generic {k} bf16")
    with load(params, tmp_path, "fp8w", "c") as m:
        check_reduced(run(m, X), params, X, "e4m3", "bf16", f"generic {k} fp8w", tol=(2e-3, 1.5e-2, 2e-2))
    for fmt, tag in (("int8", "d"), ("fp8", "e")):
        oracle_fmt, worst, typical = ROW_GATES[fmt]
        with load(params, tmp_path, fmt, tag) as m:
            check_rows_on_rounded(run(m, X), params, X, oracle_fmt, f"generic {k} {fmt}", worst=worst,
                                  typical=typical if B >= 50 else (0.0, 1.0))
