"""The 200-feature shape's two tilings on the GPU.

FP32, BF16, both FP8 forms and MXFP4 run this shape at eight waves per workgroup with the
aggregate mask kept in LDS and the step masks stored from registers; a model whose final
map leaves too little LDS for that falls back to the four-wave kernel of the same precision
(in FP32 at D = 200 and n_d = 64, beyond 18 outputs).  INT8 and the 8- and 6-bit MX forms
run at four waves.  Both kernels are checked against the FP64 oracle with the FP32 gates
of the small models (logits 1e-5 relative, masks 1e-6 times max(1, gamma^(S-1) / 2)), and
the eight-wave path for optional step masks, row independence and D not a multiple of 4
(the per-float stores)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import tabnet as oracle  # noqa: E402
from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402
from paper_2510_19689_amd.synth import TabNetConfig  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")


def model(cfg, seed, prec, tmp_path, tag="m"):
    params = synth.make_params(cfg, seed)
    path = str(tmp_path / f"{tag}.tnw")
    synth.write_weights(params, path)
    return params, tb.Model(path, prec)


def run(m, X, with_steps=True):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    lo, ag, ms = m.outputs(X.shape[0], with_steps)
    for t in (lo, ag, ms):
        if t is not None:
            t.fill_(float("nan"))
    m.forward_into(Xd, lo, ag, ms)
    torch.cuda.synchronize()
    return lo.cpu().numpy(), ag.cpu().numpy(), None if ms is None else ms.cpu().numpy()


@pytest.mark.parametrize("n_out", [3, 24])
def test_eight_and_four_wave_kernels_match_oracle(tmp_path, n_out):
    """n_out = 3 runs the eight-wave kernel, n_out = 24 the four-wave fallback (FP32)."""
    cfg = TabNetConfig(D=200, n_d=64, n_a=64, n_steps=3, n_shared=2, n_indep=1, n_out=n_out, gamma=1.3)
    params, m = model(cfg, 7100 + n_out, "fp32", tmp_path)
    X = synth.make_normal_inputs(130, cfg.D, 7200 + n_out)
    _say(f"case 200-feature fp32 n_out={n_out}")
    with m:
        lo, ag, ms = run(m, X)
    rlo, rag, rms = oracle.forward(params, X)
    rel = float((np.abs(lo - rlo).max(1) / np.maximum(np.abs(rlo).max(1), 1e-2)).max())
    mtol = 1e-6 * max(1.0, cfg.gamma ** (cfg.n_steps - 1) / 2)
    _say(n_out, "logit_rel", rel, "agg", np.abs(ag - rag).max(), "step", np.abs(ms - rms).max())
    assert rel <= 1e-5
    assert np.abs(ag - rag).max() <= mtol and np.abs(ms - rms).max() <= mtol


@pytest.mark.parametrize("D", [197, 200])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "fp8w", "mxfp4", "int8"])
def test_optional_step_masks_and_rows_independent(tmp_path, D, prec):
    """Without step masks the logits and the aggregate are bit-identical to the run with
    them; a row's outputs are the same in any sub-batch and on every run."""
    cfg = TabNetConfig(D=D, n_d=64, n_a=64, n_steps=3, n_shared=2, n_indep=1, n_out=3, gamma=1.5)
    params, m = model(cfg, 7300 + D, prec, tmp_path)
    X = synth.make_normal_inputs(333, D, 7400 + D)
    _say(f"case 200-feature {prec} D={D}")
    with m:
        full = run(m, X)
        again = run(m, X)
        nomask = run(m, X, with_steps=False)
        parts = [(lo_, hi_, run(m, X[lo_:hi_])) for lo_, hi_ in ((0, 1), (15, 17), (100, 333), (320, 333))]
    for u, v in zip(full, again):
        np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(nomask[0], full[0])
    np.testing.assert_array_equal(nomask[1], full[1])
    assert nomask[2] is None
    for lo_, hi_, p in parts:
        np.testing.assert_array_equal(p[0], full[0][lo_:hi_])
        np.testing.assert_array_equal(p[1], full[1][lo_:hi_])
        np.testing.assert_array_equal(p[2], full[2][:, lo_:hi_])
    assert np.isfinite(full[2]).all() and (full[2] >= 0).all()
    assert np.abs(full[2].sum(-1) - 1).max() <= 2e-5
