"""Pins for the oracle's bfloat16 / E4M3FN rounding against torch's CPU casts."""
import numpy as np
import torch

from oracle.rounding import round_bf16, round_e4m3


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 2000), rng.normal(0, 1e4, 2000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.0e-5])]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x.astype(np.float64)), ref)


def test_e4m3_matches_torch_cast_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(0, 0.01, 5000), rng.normal(0, 1, 5000),
                        np.array([0.0, 448.0, -448.0, 2 ** -6, 2 ** -9, 1.5 * 2 ** -9, 0.0625 * 17])])
    x = x.astype(np.float32)
    ref = torch.tensor(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_e4m3(x.astype(np.float64)), ref)


def test_e4m3_saturates():
    np.testing.assert_array_equal(round_e4m3(np.array([500.0, -1e6, 449.0])), [448.0, -448.0, 448.0])


def test_grids():
    # bf16 keeps 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    # e4m3 keeps 4 significant bits: 1 + 2^-4 ties to 1.0, 1 + 3*2^-4 ties to 1.25
    assert round_e4m3(np.array([1 + 2 ** -4]))[0] == 1.0
    assert round_e4m3(np.array([1 + 3 * 2 ** -4]))[0] == 1.25


# ---- symmetric INT8 (one scale per row) ----
from oracle.rounding import quantise_int8_rows, round_int8_rows  # noqa: E402


def _int8_inputs():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(0, 1, (300, 64)), rng.uniform(-3e-3, 3e-3, (50, 64)),
                        rng.standard_cauchy((50, 64))])
    x[5] = 0.0                       # an all-zero row
    x[6, :] = 2.5                    # a constant row
    x[7, 3] = -9.0                   # negative maximum
    return x


def test_int8_codes_match_torch_quantize_per_channel():
    """torch's per-channel qint8 quantiser (round half to even, zero point 0) is an
    independent implementation of c = round(x / s) for the same scales."""
    x = _int8_inputs().astype(np.float32)       # torch quantises float32 tensors
    codes, scale = quantise_int8_rows(x.astype(np.float64))
    ref = torch.quantize_per_channel(torch.tensor(x), torch.tensor(scale[:, 0]), torch.zeros(len(x), dtype=torch.long),
                                     0, torch.qint8).int_repr().numpy().astype(np.int64)
    # torch divides in its own precision: allow disagreement only where x / s lies within
    # 2e-5 of a half-integer (a rounding boundary)
    t = x / scale
    near_tie = np.abs(np.abs(t - np.floor(t)) - 0.5) < 2e-5
    assert (codes[~near_tie] == ref[~near_tie]).all()
    assert near_tie.mean() < 1e-3


def test_int8_closed_forms():
    x = _int8_inputs()
    codes, scale = quantise_int8_rows(x)
    assert codes.dtype == np.int64 and scale.shape == (len(x), 1)
    assert np.abs(codes).max() <= 127
    nz = np.abs(x).max(1) > 0
    # the row maximum maps to +-127 exactly; every other code is within half a step
    assert (np.abs(codes[nz]).max(1) == 127).all()
    np.testing.assert_allclose(scale[nz, 0], np.abs(x[nz]).max(1) / 127, rtol=0, atol=0)
    assert (np.abs(x - codes * scale) <= scale / 2 * (1 + 1e-12)).all()
    # zero row: zero codes, unit scale; constant row: all 127
    assert (codes[5] == 0).all() and scale[5, 0] == 1.0
    assert (codes[6] == 127).all() and codes[7, 3] == -127
    # odd symmetry and scale invariance by powers of two
    c2, _ = quantise_int8_rows(-x)
    assert (c2 == -codes).all()
    c3, s3 = quantise_int8_rows(x * 8.0)
    assert (c3 == codes).all() and np.array_equal(s3[nz], scale[nz] * 8.0)
    np.testing.assert_array_equal(round_int8_rows(x), codes * scale)


def test_int8_ties_to_even():
    # scale 1 (row max 127): the codes of half-integers go to the even neighbour
    x = np.array([[127.0, 0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 126.5, 3.25]])
    codes, scale = quantise_int8_rows(x)
    assert scale[0, 0] == 1.0
    assert codes.tolist() == [[127, 0, 2, 2, 0, -2, -2, 126, 3]]


def test_int8_gemm_option_matches_torch_dequantised_product():
    """The oracle's INT8 GEMM operands (weights per output channel, inputs per row) against
    torch's quantise / dequantise with the same scales, multiplied in float64.  The batch
    norm is the identity (var + eps = 1 exactly), so W' = W; the operands lie off the
    INT8 grid, and float32 so that torch can quantise them."""
    from oracle import tabnet as ot
    rng = np.random.default_rng(11)
    u = rng.normal(0, 1, (40, 24)).astype(np.float32)
    W = rng.normal(0, 0.3, (10, 24)).astype(np.float32)
    eps = 2.0 ** -10
    bn = {"gamma": np.ones(10), "beta": np.zeros(10), "mean": np.zeros(10), "var": np.full(10, 1 - eps)}
    got = ot._fc_bn(u.astype(np.float64), W, bn, eps, weights="int8", acts="int8")

    def tq(a):
        sc = np.abs(a.astype(np.float64)).max(1) / 127
        q = torch.quantize_per_channel(torch.tensor(a), torch.tensor(sc), torch.zeros(len(a), dtype=torch.long), 0,
                                       torch.qint8)
        return q.int_repr().numpy().astype(np.float64) * sc[:, None]
    ref = tq(u) @ tq(W).T
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_int8_gemm_within_error_bound():
    """With any batch norm, the INT8 product stays within the bound that half a step per
    operand gives: |d| <= sum_k (|du_k| |w_k| + |u_k| |dw_k| + |du_k| |dw_k|)."""
    from oracle import tabnet as ot
    rng = np.random.default_rng(12)
    u = rng.normal(0, 1, (40, 24))
    W = rng.normal(0, 0.3, (10, 24))
    bn = {"gamma": rng.uniform(0.5, 1.5, 10), "beta": rng.normal(0, 0.1, 10),
          "mean": rng.normal(0, 0.1, 10), "var": rng.uniform(0.5, 2.0, 10)}
    eps = 1e-5
    got = ot._fc_bn(u, W, bn, eps, weights="int8", acts="int8")
    s = bn["gamma"] / np.sqrt(bn["var"] + eps)
    Wf = W * s[:, None]
    exact = u @ Wf.T + (bn["beta"] - s * bn["mean"])
    su = np.abs(u).max(1, keepdims=True) / 127
    sw = np.abs(Wf).max(1, keepdims=True) / 127
    K = u.shape[1]
    bound = (su / 2) * np.abs(Wf).sum(1)[None, :] + np.abs(u).sum(1)[:, None] * (sw / 2).T + K * (su / 2) * (sw / 2).T
    assert (np.abs(got - exact) <= bound * (1 + 1e-9)).all()
    assert np.abs(got - exact).max() > 0          # the operands really were rounded


def test_e4m3_row_scaled_inputs_match_torch():
    """The oracle's E4M3 GEMM-input option (one scale per row, max |u| / 448) against
    torch's E4M3 cast of u / s: the largest entry of each row lands on 448."""
    from oracle import tabnet as ot
    rng = np.random.default_rng(13)
    u = rng.normal(0, 1, (64, 40)) * rng.uniform(1e-3, 1e3, (64, 1))
    u[7] = 0.0
    got = ot._round_acts(u, "e4m3")
    amax = np.abs(u).max(1, keepdims=True)
    sc = np.where(amax > 0, amax / 448.0, 1.0)
    ref = torch.tensor(u / sc, dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64).numpy() * sc
    np.testing.assert_array_equal(got, ref)
    nz = amax[:, 0] > 0
    np.testing.assert_allclose(np.abs(got[nz]).max(1), amax[nz, 0], rtol=4e-16, atol=0)   # 448 (max / 448)
    assert (got[7] == 0).all()
