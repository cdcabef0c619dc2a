"""Every row of the benchmarked launches against the FP64 oracle (GPU).

The Adult-shaped model at its full batch (65,536 rows, 5 steps, step masks on) in every
precision, and the 200-feature model at its full batch (1,048,576 rows, 7 steps) in FP32,
BF16 and FP8: one launch each, in the configuration the benchmark times, then every row
against the oracle, chunk by chunk in worker processes (tests/fullsize.py).  The gates
are those of the target where the arithmetic meets them; each departure is a documented
deviation with its measured size (GATES below, and the tolerance table of the design
notes).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402
import fullsize  # noqa: E402

pytestmark = pytest.mark.gpu

MX_FORMATS = ["mxfp8", "mxfp8_e5m2", "mxfp6", "mxfp6_e3m2", "mxfp4"]
# oracle rounding of each precision's GEMM operands (weights, acts)
ROUNDING = {"bf16": ("bf16", "bf16"), "fp8": ("e4m3", "e4m3"), "fp8w": ("e4m3", "bf16"), "int8": ("int8", "int8"),
            **{f: (f, f) for f in MX_FORMATS}}


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    if not os.path.exists(tb.LIB_PATH):
        pytest.fail("libtabnet.so not built")


def launch_all(params, X, precs, tmp_path):
    """One full-batch launch per precision (step masks on); outputs stay on the GPU."""
    path = str(tmp_path / "m.tnw")
    synth.write_weights(params, path)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    outs = {}
    for p in precs:
        _say(f"launch {p} rows={X.shape[0]}")
        with tb.Model(path, p) as m:
            lo, ag, ms = m.outputs(X.shape[0], True)
            for t in (lo, ag, ms):
                t.fill_(float("nan"))
            m.forward_into(Xd, lo, ag, ms)
            torch.cuda.synchronize()
        outs[p] = (lo, ag, ms)
    del Xd
    return outs


def fetcher(outs):
    def fetch(lo, hi):
        return {p: (a[lo:hi].cpu().numpy(), b[lo:hi].cpu().numpy(), c[:, lo:hi].cpu().numpy())
                for p, (a, b, c) in outs.items()}
    return fetch


def invariants(outs, tag):
    """On the device, every row: finite, non-negative, each step mask sums to 1 and each
    aggregate mask sums to 1 or is a zero row."""
    for p, (lo, ag, ms) in outs.items():
        assert bool(torch.isfinite(lo).all()) and bool(torch.isfinite(ag).all()), (tag, p)
        assert bool(torch.isfinite(ms).all()) and bool((ms >= 0).all()) and bool((ag >= 0).all()), (tag, p)
        assert float((ms.sum(-1) - 1).abs().max()) <= 2e-5, (tag, p)
        sa = ag.sum(-1)
        assert bool((((sa - 1).abs() <= 2e-5) | (sa == 0)).all()), (tag, p)


def ratios(errs, tag):
    for name in errs:
        if name.endswith("@op"):
            p = name[:-3]
            for m in ("step_l1", "logit_abs", "agg_l1"):
                r = errs[name][m] / np.maximum(errs[p + "@format"][m], 1e-6)
                q = np.quantile(r, [0.5, 0.9, 0.99, 0.999, 1.0])
                _say(f"RATIO {tag} {p} {m} op/format q50,90,99,99.9,max", np.round(q, 4).tolist(),
                     "rows op>1e-5:", float((errs[name][m] > 1e-5).mean()))


def report(name, e):
    s = fullsize.summary(e)
    _say(name, {k: (round(v, 9) if isinstance(v, float) else v) for k, v in s.items()})
    return s


def test_adult108_every_row_every_precision(tmp_path):
    params, X = synth.workload("adult108")
    assert X.shape == (65536, 108)
    precs = ["fp32", "bf16", "fp8", "fp8w", "int8"] + MX_FORMATS
    outs = launch_all(params, X, precs, tmp_path)
    invariants(outs, "adult108")
    checks = ([(p, p, None, None) for p in precs] + [(p + "@op", p, *ROUNDING[p]) for p in precs if p != "fp32"]
              + [(p + "@format", fullsize.OracleRounded(*ROUNDING[p]), None, None) for p in precs if p != "fp32"])
    errs = fullsize.all_rows(params, X, fetcher(outs), checks, chunk=4096, say=_say)
    S = {name: report(f"adult108 {name}", e) for name, e in errs.items()}
    ratios(errs, "adult108")
    failures = gate_failures(errs, S, "adult108", params["config"])
    assert not failures, failures


def test_wide200_every_row_fp32_bf16_fp8(tmp_path):
    """The 200-feature model at its full batch in FP32, BF16 and both FP8 readings (E4M3 on
    both GEMM operands with row scales; E4M3 weights with BF16 inputs)."""
    params, X = synth.workload("wide200")
    assert X.shape == (1048576, 200)
    precs = ["fp32", "bf16", "fp8", "fp8w"]
    outs = launch_all(params, X, precs, tmp_path)
    invariants(outs, "wide200")
    checks = [(p, p, None, None) for p in precs]
    errs = fullsize.all_rows(params, X, fetcher(outs), checks, chunk=8192, say=_say)
    S = {name: report(f"wide200 {name}", e) for name, e in errs.items()}
    all_errs = dict(errs)
    # the operand-rounded references on the first 65,536 rows
    n = 65536
    sub = {p: tuple(t[:n] if t.dim() < 3 else t[:, :n] for t in outs[p]) for p in ("bf16", "fp8", "fp8w")}
    checks = ([(p + "@op", p, *ROUNDING[p]) for p in sub]
              + [(p + "@format", fullsize.OracleRounded(*ROUNDING[p]), None, None) for p in sub])
    errs = fullsize.all_rows(params, X[:n], fetcher(sub), checks, chunk=4096, say=_say)
    S.update({name: report(f"wide200[:{n}] {name}", e) for name, e in errs.items()})
    ratios(errs, "wide200")
    all_errs.update(errs)
    failures = gate_failures(all_errs, S, "wide200", params["config"])
    assert not failures, failures


# Gates against plain FP64, on every row (metric -> bound; "argmax" -> least agreement).
# Where the target's bound is below what the number format itself allows, the bound is the
# format's measured error with a margin, and the design notes list it as a deviation:
#   FP32 masks: 1e-6 scaled by the prior's growth max(1, gamma^(S-1) / 2) (an FP32 score of
#     size 2^k carries a rounding unit of 2^(k-24)); measured 1.2e-6 (Adult-shaped, bound
#     2.5e-6) and 1.8e-6 (200 features, bound 2.4e-6).
#   BF16 step masks: FP64 on the same bf16-rounded operands already reaches a step-mask L1 of
#     2.0e-2 (Adult-shaped) and 1.2e-2 (200 features); the kernel's worst rows equal it.
#   FP8, INT8, MX: the formats' own errors (FP64 on their operands against plain FP64).
FP64_GATES = {
    "bf16": {"logit_abs": 2e-2, "agg_l1": 1e-2, "step_l1": 2.5e-2, "argmax": 0.999},
    "fp8": {"logit_abs": 2e-2, "agg_l1": 0.1, "step_l1": 0.4, "argmax": 0.999},
    "fp8w": {"logit_abs": 2e-2, "agg_l1": 0.1, "step_l1": 0.4, "argmax": 0.999},
    "int8": {"logit_abs": 2e-2, "agg_l1": 0.06, "step_l1": 0.3, "argmax": 0.999},
    "mxfp8": {"logit_abs": 2e-2, "agg_l1": 0.1, "step_l1": 0.5, "argmax": 0.999},
    "mxfp8_e5m2": {"logit_abs": 5e-2, "agg_l1": 0.2, "step_l1": 0.85, "argmax": 0.999},
    "mxfp6": {"logit_abs": 2e-2, "agg_l1": 0.12, "step_l1": 0.45, "argmax": 0.999},
    "mxfp6_e3m2": {"logit_abs": 5e-2, "agg_l1": 0.2, "step_l1": 0.85, "argmax": 0.999},
    "mxfp4": {"logit_abs": 6e-2, "agg_l1": 0.4, "step_l1": 1.6, "argmax": 0.999},
}
# Formats whose matrix instruction sums their products exactly (INT32, or exactly in FP32):
# a row moves from FP64 on the same operands only where an FP32 GEMM input lands on the
# other side of a rounding boundary than its FP64 value (a code flip).
EXACT_SUMS = ("int8", "mxfp6", "mxfp4")


def gate_failures(errs, S, tag, cfg):
    """Every gate that fails, as text."""
    out = []

    def bound(name, metric, v, b, low=False):
        if (v < b) if low else (v > b):
            out.append(f"{tag} {name} {metric} = {v:.3g} (gate {b:g})")

    for name, s in S.items():
        if name == "fp32":
            mtol = 1e-6 * max(1.0, cfg.gamma ** (cfg.n_steps - 1) / 2)
            bound(name, "logit_rel", s["logit_rel"], 1e-5)
            bound(name, "agg_abs", s["agg_abs"], mtol)
            bound(name, "step_abs", s["step_abs"], mtol)
        elif name in FP64_GATES:
            for metric, b in FP64_GATES[name].items():
                bound(name, metric, s[metric], b, low=metric == "argmax")
        elif name.endswith("@op"):
            # Row by row against FP64 on the same rounded operands: a row may move by code
            # flips, each a part of the format's own error on that row, so each row's
            # departure is bounded by its own format error (measured at most 2.2x in the
            # step masks and 1.4x in the aggregate, over every format and both models); a
            # wrong index, scale or row moves a row by far more than its format error.
            p = name[:-3]
            e, f = errs[name], errs[p + "@format"]
            r_step = float(np.max(e["step_l1"] - 2.5 * f["step_l1"]))
            r_agg = float(np.max(e["agg_l1"] - 2.0 * f["agg_l1"]))
            bound(name, "step_l1 - 2.5 format", r_step, 1e-5)
            bound(name, "agg_l1 - 2 format", r_agg, 1e-5)
            if p in EXACT_SUMS:
                bound(name, "rows moved (step L1 > 1e-5)", float((e["step_l1"] > 1e-5).mean()), 0.01)
            if p == "bf16":
                bound(name, "step_l1", s["step_l1"], 1e-2)
                bound(name, "logit_abs", s["logit_abs"], 1e-3)
    return out
