"""Pins for the oracle's OCP MX block formats (MXFP8 = E4M3 or E5M2 elements, MXFP6 =
E2M3 or E3M2 elements, MXFP4 = E2M1 elements, one power-of-two scale per block of 32;
CPU only)."""
import numpy as np
import pytest
import torch

from oracle.rounding import (E2M1_MAX, E2M3_MAX, E3M2_MAX, E5M2_MAX, mx_scale_exponent, round_e2m1, round_e2m3,
                             round_e3m2, round_e4m3, round_e5m2, round_mx_rows)
from oracle import tabnet as ot

FMTS = ["mxfp8", "mxfp8_e5m2", "mxfp6", "mxfp6_e3m2", "mxfp4"]
ROUND = {"mxfp8": round_e4m3, "mxfp8_e5m2": round_e5m2, "mxfp6": round_e2m3, "mxfp6_e3m2": round_e3m2,
         "mxfp4": round_e2m1}
# from the element formats' definitions: (emax, largest normal, stored mantissa bits)
ELEM = {"mxfp8": (8, 448.0, 3), "mxfp8_e5m2": (15, 57344.0, 2), "mxfp6": (2, 7.5, 3), "mxfp6_e3m2": (4, 28.0, 2),
        "mxfp4": (2, 6.0, 1)}


def e2m1_table():
    """All 16 FP4 E2M1 codes decoded from the bit fields: sign, 2-bit exponent (bias 1),
    1-bit mantissa; exponent 0 is subnormal (m / 2)."""
    vals = []
    for c in range(16):
        s = -1.0 if c & 8 else 1.0
        e, m = (c >> 1) & 3, c & 1
        vals.append(s * (m / 2.0 if e == 0 else (1 + m / 2.0) * 2.0 ** (e - 1)))
    return np.array(vals)


def test_e2m1_grid_and_brute_force_rounding():
    table = e2m1_table()
    assert sorted(set(np.abs(table))) == [0, 0.5, 1, 1.5, 2, 3, 4, 6]
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-8, 8, 5000), np.arange(-7, 7.01, 0.25), [0.0, 100.0, -100.0]])
    got = round_e2m1(x)
    for v, g in zip(x, got):
        a = min(abs(v), E2M1_MAX)
        d = np.abs(table[:8] - a)
        best = np.flatnonzero(d == d.min())
        code = best[0] if len(best) == 1 else [b for b in best if b % 2 == 0][0]   # ties: even code
        assert g == np.copysign(table[code], v), (v, g, table[code])


def e2m3_table():
    """All 32 FP6 E2M3 codes decoded from the bit fields: sign, 2-bit exponent (bias 1),
    3-bit mantissa; exponent 0 is subnormal (m / 8)."""
    vals = []
    for c in range(32):
        s = -1.0 if c & 32 else 1.0
        e, m = (c >> 3) & 3, c & 7
        vals.append(s * (m / 8.0 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 1)))
    return np.array(vals)


def test_e2m3_grid_and_brute_force_rounding():
    table = e2m3_table()
    assert max(table) == E2M3_MAX and len(set(np.abs(table))) == 32
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.uniform(-9, 9, 5000), np.arange(-8, 8.01, 1 / 16), [0.0, 100.0, -100.0]])
    got = round_e2m3(x)
    pos = table[:32]
    for v, g in zip(x, got):
        a = min(abs(v), E2M3_MAX)
        d = np.abs(pos - a)
        best = np.flatnonzero(d == d.min())
        code = best[0] if len(best) == 1 else [b for b in best if b % 2 == 0][0]   # ties: even code
        assert g == np.copysign(pos[code], v), (v, g, pos[code])


def e3m2_table():
    """All 32 FP6 E3M2 magnitudes decoded from the bit fields: 3-bit exponent (bias 3),
    2-bit mantissa; exponent 0 is subnormal (m / 4 * 2^-2)."""
    vals = []
    for c in range(32):
        e, m = c >> 2, c & 3
        vals.append(m / 16.0 if e == 0 else (1 + m / 4.0) * 2.0 ** (e - 3))
    return np.array(vals)


def test_e3m2_grid_and_brute_force_rounding():
    pos = e3m2_table()
    assert pos.max() == E3M2_MAX and len(set(pos)) == 32 and pos[1] == 1 / 16 and pos[4] == 0.25
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-33, 33, 5000), rng.uniform(-0.6, 0.6, 3000), np.arange(-30, 30.01, 1 / 32),
                        [0.0, 100.0, -100.0]])
    got = round_e3m2(x)
    for v, g in zip(x, got):
        a = min(abs(v), E3M2_MAX)
        d = np.abs(pos - a)
        best = np.flatnonzero(d == d.min())
        code = best[0] if len(best) == 1 else [b for b in best if b % 2 == 0][0]   # ties: even code
        assert g == np.copysign(pos[code], v), (v, g, pos[code])


def test_e5m2_matches_torch_and_saturates():
    """torch's float8_e5m2 decodes every code and rounds float32 values to nearest even;
    its cast does not saturate (from 61440 up it gives inf), the oracle's does."""
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e5m2).to(torch.float64).numpy()
    fin = np.unique(codes[np.isfinite(codes)])
    np.testing.assert_array_equal(round_e5m2(fin), fin)            # every finite code is on the grid
    assert fin.max() == E5M2_MAX and np.abs(fin[fin != 0]).min() == 2.0 ** -16
    mid = (fin[:-1] + fin[1:]) / 2                                  # ties between neighbours
    rng = np.random.default_rng(7)
    n = 20000
    wide = np.ldexp(rng.uniform(1, 2, n), rng.integers(-20, 17, n)) * rng.choice([-1.0, 1.0], n)
    x = np.concatenate([wide, mid, fin]).astype(np.float32).astype(np.float64)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e5m2).to(torch.float64).numpy()
    ok = np.isfinite(ref)
    np.testing.assert_array_equal(round_e5m2(x[ok]), ref[ok])
    assert (np.abs(x[~ok]) >= 61440).all() and (~ok).any()
    np.testing.assert_array_equal(round_e5m2(np.array([61440.0, 1e6, -7e4])), [E5M2_MAX, E5M2_MAX, -E5M2_MAX])


def test_scale_exponent_ocp_rule():
    amax = np.array([1.0, 1.5, 2.0, 448.0, 500.0, 2.0 ** -20, 0.0, 3.0e38, 1e-40])
    X8 = mx_scale_exponent(amax, "mxfp8")
    X4 = mx_scale_exponent(amax, "mxfp4")
    np.testing.assert_array_equal(X8[:6], [-8, -8, -7, 0, 0, -28])
    np.testing.assert_array_equal(X4[:6], [-2, -2, -1, 6, 6, -22])
    assert X8[6] == 0 and X4[6] == 0
    assert X8[7] == 127 - 8 and X8[8] == -126     # clamped below
    # the block maximum lands in [2^emax, 2^(emax + 1)) after scaling
    for fmt in FMTS:
        emax = ELEM[fmt][0]
        a = np.abs(np.random.default_rng(2).normal(0, 5, 1000)) + 1e-3
        r = a / np.ldexp(1.0, mx_scale_exponent(a, fmt))
        assert ((r >= 2.0 ** emax) & (r < 2.0 ** (emax + 1))).all()


def e4m3_table():
    """The non-negative finite FP8 E4M3 (OCP E4M3FN) values in code order, decoded from the
    bit fields: 4-bit exponent (bias 7), 3-bit mantissa, exponent 0 subnormal (m / 8 *
    2^-6); code 0x7f (all ones) is NaN and has no value."""
    vals = []
    for c in range(0x7f):
        e, m = c >> 3, c & 7
        vals.append(m / 8.0 * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


def e5m2_table():
    """The non-negative finite FP8 E5M2 values in code order: 5-bit exponent (bias 15),
    2-bit mantissa, exponent 0 subnormal (m / 4 * 2^-14); exponent 31 holds inf and NaN."""
    vals = []
    for c in range(0x7c):
        e, m = c >> 2, c & 3
        vals.append(m / 4.0 * 2.0 ** -14 if e == 0 else (1 + m / 4.0) * 2.0 ** (e - 15))
    return np.array(vals)


def element_table(fmt):
    return {"mxfp8": e4m3_table, "mxfp8_e5m2": e5m2_table, "mxfp6": lambda: e2m3_table()[:32],
            "mxfp6_e3m2": e3m2_table, "mxfp4": lambda: e2m1_table()[:8]}[fmt]()


def nearest_code(table, v):
    """Value of the code nearest to v in the ascending table of non-negative values, ties
    to the even code, saturating at the largest entry; the sign is carried over."""
    a = min(abs(v), table[-1])
    d = [abs(t - a) for t in table]
    lo = min(d)
    best = [i for i, x in enumerate(d) if x == lo]
    code = best[0] if len(best) == 1 else [i for i in best if i % 2 == 0][0]
    return -table[code] if v < 0 else table[code]


def brute_mx(x, fmt):
    """From the OCP MX definition alone, element by element (pure Python over a small
    matrix): the element's block is the 32 consecutive elements k // 32 = j // 32; the
    block's shared exponent is the X with 2^(X + emax) <= max|block| < 2^(X + emax + 1),
    found by stepping X, clamped to the E8M0 range [-127 + 1, 127]; the element is the
    format's code nearest to x / 2^X (ties to even), times 2^X."""
    rows, K = x.shape
    out = np.zeros_like(x)
    emax = ELEM[fmt][0]
    table = element_table(fmt)
    for r in range(rows):
        for j in range(K):
            members = [k for k in range(K) if k // 32 == j // 32]
            m = max(abs(x[r, k]) for k in members)
            if m == 0:
                continue
            X = 0
            while 2.0 ** (X + emax) > m:
                X -= 1
            while 2.0 ** (X + emax + 1) <= m:
                X += 1
            X = min(max(X, -126), 127)
            out[r, j] = nearest_code(table, x[r, j] / 2.0 ** X) * 2.0 ** X
    return out


def test_element_tables_decode_the_formats():
    assert e4m3_table()[-1] == 448.0 and e4m3_table()[1] == 2.0 ** -9 and len(set(e4m3_table())) == 127
    assert e5m2_table()[-1] == E5M2_MAX and e5m2_table()[1] == 2.0 ** -16 and len(set(e5m2_table())) == 124
    for fmt in FMTS:
        t = element_table(fmt)
        assert (np.diff(t) > 0).all() and t[0] == 0.0 and t[-1] == ELEM[fmt][1]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("K", [8, 35, 64, 100, 108])
def test_round_mx_rows_matches_brute_force(fmt, K):
    rng = np.random.default_rng(K)
    x = rng.normal(0, 1, (5, K)) * np.array([[1.0], [1e-3], [300.0], [1.0], [1.0]])
    x[3, :] = 0.0
    x[3, min(5, K - 1)] = -2.5
    x[4, ::7] *= 40.0            # blocks of very different ranges side by side
    np.testing.assert_array_equal(round_mx_rows(x, fmt), brute_mx(x, fmt))


@pytest.mark.parametrize("fmt", FMTS)
def test_blocks_are_consecutive_32(fmt):
    """A large value changes the scale of its own 32-element block only."""
    x = np.random.default_rng(9).normal(0, 1, (1, 100))
    big = x.copy()
    big[0, 40] = 1e4
    a, b = round_mx_rows(x, fmt), round_mx_rows(big, fmt)
    changed = np.flatnonzero(a[0] != b[0])
    assert changed.min() >= 32 and changed.max() < 64 and 40 in changed


def test_mxfp8_elements_match_torch_e4m3_and_saturate():
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (50, 128))
    got = round_mx_rows(x, "mxfp8")
    for b in range(4):
        cols = slice(32 * b, 32 * b + 32)
        X = mx_scale_exponent(np.abs(x[:, cols]).max(1, keepdims=True), "mxfp8")
        sc = np.ldexp(1.0, X)
        # torch's E4M3 cast does not saturate: clamp to the largest normal first
        ref = torch.tensor(np.clip(x[:, cols] / sc, -448, 448), dtype=torch.float32)
        ref = ref.to(torch.float8_e4m3fn).to(torch.float64).numpy() * sc
        np.testing.assert_array_equal(got[:, cols], ref)
    # a block whose maximum scales into (448, 512) saturates at 448 * 2^X
    y = np.zeros((1, 32))
    y[0, 0], y[0, 1] = 500.0, 1.0
    r = round_mx_rows(y, "mxfp8")
    assert r[0, 0] == 448.0 and r[0, 1] == 1.0


@pytest.mark.parametrize("fmt", FMTS)
def test_mx_exact_on_grid_and_scale_equivariant(fmt):
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (6, 100))
    r = round_mx_rows(x, fmt)
    np.testing.assert_array_equal(round_mx_rows(r, fmt), r)            # idempotent
    np.testing.assert_array_equal(round_mx_rows(x * 2.0 ** 7, fmt), r * 2.0 ** 7)
    np.testing.assert_array_equal(round_mx_rows(-x, fmt), -r)
    # per element: within half a step of the grid at the block's scale (the step of the
    # top binade [2^emax, 2^(emax+1)) bounds all), or saturated at the largest normal
    emax, vmax, mbits = ELEM[fmt]
    for b in range(4):
        cols = slice(32 * b, 32 * b + 32)
        sc = np.ldexp(1.0, mx_scale_exponent(np.abs(x[:, cols]).max(1, keepdims=True), fmt))
        step = sc * 2.0 ** (emax - mbits)
        err = np.abs(r[:, cols] - x[:, cols])
        sat = (np.abs(x[:, cols]) > vmax * sc) & (np.abs(r[:, cols]) == vmax * sc)
        assert ((err <= step / 2 * (1 + 1e-12)) | sat).all()


def test_mx_gemm_option_uses_both_operands_and_attention_half_from_zero(monkeypatch):
    """_fc_bn rounds the input rows and the weight rows in blocks of the same 32 K
    positions; the attentive GEMM's input is the attention half alone, so its blocks
    start at its own first column."""
    rng = np.random.default_rng(5)
    u = rng.normal(0, 1, (7, 40))
    W = rng.normal(0, 0.3, (5, 40))
    eps = 2.0 ** -10
    bn = {"gamma": np.ones(5), "beta": np.zeros(5), "mean": np.zeros(5), "var": np.full(5, 1 - eps)}
    for fmt in ("mxfp8", "mxfp4"):
        got = ot._fc_bn(u, W, bn, eps, weights=fmt, acts=fmt)
        ref = brute_mx(u, fmt) @ brute_mx(W, fmt).T
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
    seen = []
    real = ot._round_acts

    def spy(u_, mode):
        seen.append(u_.copy())
        return real(u_, mode)
    monkeypatch.setattr(ot, "_round_acts", spy)
    from paper_2510_19689_amd import synth
    p, X = synth.workload("adult108", rows=3)
    cfg = p["config"]
    _, _, _, inter = ot.forward(p, X, weights="mxfp8", acts="mxfp8", internals=True)
    widths = [s_.shape[1] for s_ in seen]
    # per pass: the first layer on D features, the later ones on N channels; per step the
    # attentive GEMM on the n_a channels of the attention half
    L = cfg.n_shared + cfg.n_indep
    assert widths.count(cfg.D) == cfg.n_steps + 1
    assert widths.count(cfg.n_d + cfg.n_a) == (cfg.n_steps + 1) * (L - 1)
    assert widths.count(cfg.n_a) == cfg.n_steps
