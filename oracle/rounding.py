"""Round-to-nearest-even onto the reduced-precision grids, written from the formats'
definitions (test infrastructure; never on the product path).

The paper names reduced-precision arithmetic, beside kernel fusion, as a next step for
its TabNet inference (Sec. VI-D).  The oracle can round GEMM operands the way
a reduced-precision path defines them, so that a reduced-precision GPU result can be
compared both with exact FP64 TabNet and with FP64 TabNet on the rounded operands.

  bfloat16      : 8 significant bits (1 implicit + 7 stored), float32's exponent range.
  float8 E4M3FN : 4 significant bits (1 implicit + 3 stored), exponent bias 7, smallest
                  normal 2^-6, subnormal step 2^-9, largest finite 448, no infinities;
                  out-of-range values saturate to +-448 here.
  int8, symmetric: the paper's own example of reduced precision is FP32 to INT8
                  (Sec. VI-D).  A vector v (one weight row, or one row of a GEMM input)
                  is stored as integer codes c in [-127, 127] and one scale
                  s = max|v| / 127 (s = 1 for an all-zero vector): c = round(v / s), ties
                  to even, and v is read back as c * s.  The largest |v| maps to +-127
                  exactly, so no code needs clamping and -128 is never used.
  MX block formats (OCP Microscaling v1.0): blocks of 32 elements share one power-of-two
                  scale 2^X (an E8M0 byte) with X = floor(log2 max|v|) - emax_elem, and
                  each element is v / 2^X rounded to nearest even in the element format,
                  saturating at its largest normal.  Elements: E4M3 (MXFP8, emax 8, max
                  448), E5M2 (MXFP8 in its other element form: exponent bias 15, 2 stored
                  mantissa bits, smallest normal 2^-14, subnormal step 2^-16, emax 15,
                  max 57344), E2M3 (MXFP6, emax 2, step 1/8 below 1, 3 stored mantissa
                  bits from 1 up, max 7.5), E3M2 (MXFP6 in its other form: exponent bias
                  3, 2 stored mantissa bits, smallest normal 1/4, step 1/16 below it,
                  emax 4, max 28) and E2M1 (MXFP4, emax 2, grid 0, 0.5, 1, 1.5, 2, 3, 4,
                  6).  X is
                  clamped to [-126, 127] (a block of zeros takes X = 0).  Blocks are 32
                  consecutive elements of the vector along the reduction axis K, the
                  first starting at element 0; when K is not a multiple of 32 the last
                  block holds the remaining elements (as if padded with zeros, which
                  change neither the maximum nor any element).
"""
from __future__ import annotations

import numpy as np


def _round_sig(x: np.ndarray, bits: int) -> np.ndarray:
    """Round float64 x to `bits` significant bits, ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m * 2^e with 0.5 <= |m| < 1
    scaled = np.ldexp(m, bits)              # |scaled| in [2^(bits-1), 2^bits)
    r = np.rint(scaled)                     # ties to even
    return np.ldexp(r, e - bits)


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    out = _round_sig(x, 8)
    return np.where(np.isfinite(x), out, x)


E4M3_MAX = 448.0


def round_e4m3(x) -> np.ndarray:
    """Nearest float8 E4M3FN value (ties to even, saturating at +-448), as float64."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    normal = _round_sig(x, 4)
    sub = np.rint(x * 2.0 ** 9) * 2.0 ** -9     # fixed 2^-9 grid below 2^-6
    out = np.where(ax < 2.0 ** -6, sub, normal)
    return np.clip(out, -E4M3_MAX, E4M3_MAX)


INT8_MAX = 127.0


def quantise_int8_rows(x):
    """Symmetric INT8 codes of every row of x (last axis): returns (codes, scales) with
    codes int64 in [-127, 127] and scales float64 of shape x.shape[:-1] + (1,)."""
    x = np.asarray(x, dtype=np.float64)
    amax = np.max(np.abs(x), axis=-1, keepdims=True)
    scale = np.where(amax > 0, amax / INT8_MAX, 1.0)
    codes = np.rint(x / scale).astype(np.int64)
    return codes, scale


def round_int8_rows(x) -> np.ndarray:
    """x with every row replaced by its symmetric INT8 reading codes * scale (float64)."""
    codes, scale = quantise_int8_rows(x)
    return codes * scale


# ---- OCP MX block formats ----
E2M1_MAX = 6.0
E2M3_MAX = 7.5
E3M2_MAX = 28.0
E5M2_MAX = 57344.0
# element format of each MX format: (emax, largest normal)
MX_BLOCK = 32   # elements per block (OCP MX)
MX_ELEMENTS = {"mxfp8": (8, E4M3_MAX), "mxfp8_e5m2": (15, E5M2_MAX), "mxfp6": (2, E2M3_MAX),
               "mxfp6_e3m2": (4, E3M2_MAX), "mxfp4": (2, E2M1_MAX)}


def round_e5m2(x) -> np.ndarray:
    """Nearest float8 E5M2 value (ties to even), saturating at +-57344, as float64.  E5M2
    has 3 significant bits from 2^-14 up (exponent bias 15) and a step of 2^-16 below."""
    x = np.asarray(x, dtype=np.float64)
    normal = _round_sig(x, 3)
    sub = np.rint(x * 2.0 ** 16) * 2.0 ** -16
    out = np.where(np.abs(x) < 2.0 ** -14, sub, normal)
    return np.clip(out, -E5M2_MAX, E5M2_MAX)


def round_e3m2(x) -> np.ndarray:
    """Nearest FP6 E3M2 value (ties to even), saturating at +-28, as float64.  E3M2 has
    3 significant bits from 1/4 up (exponent bias 3) and a step of 1/16 below 1/4."""
    x = np.asarray(x, dtype=np.float64)
    normal = _round_sig(x, 3)
    sub = np.rint(x * 16.0) / 16.0
    out = np.where(np.abs(x) < 0.25, sub, normal)
    return np.clip(out, -E3M2_MAX, E3M2_MAX)


def round_e2m3(x) -> np.ndarray:
    """Nearest FP6 E2M3 value (ties to even), saturating at +-7.5, as float64.  E2M3 has
    4 significant bits from 1 up (exponent bias 1) and a step of 1/8 below 1."""
    x = np.asarray(x, dtype=np.float64)
    normal = _round_sig(x, 4)
    sub = np.rint(x * 8.0) / 8.0
    out = np.where(np.abs(x) < 1.0, sub, normal)
    return np.clip(out, -E2M3_MAX, E2M3_MAX)


def round_e2m1(x) -> np.ndarray:
    """Nearest FP4 E2M1 value (ties to even), saturating at +-6, as float64.  E2M1 has
    2 significant bits from 1 up (exponent bias 1) and a step of 0.5 below 1."""
    x = np.asarray(x, dtype=np.float64)
    normal = _round_sig(x, 2)
    sub = np.rint(x * 2.0) / 2.0
    out = np.where(np.abs(x) < 1.0, sub, normal)
    return np.clip(out, -E2M1_MAX, E2M1_MAX)


def _round_element(v, fmt):
    return {"mxfp8": round_e4m3, "mxfp8_e5m2": round_e5m2, "mxfp6": round_e2m3, "mxfp6_e3m2": round_e3m2,
            "mxfp4": round_e2m1}[fmt](v)


def mx_scale_exponent(amax, fmt) -> np.ndarray:
    """X = floor(log2 amax) - emax_elem, clamped to [-126, 127]; 0 where amax = 0."""
    emax = MX_ELEMENTS[fmt][0]
    amax = np.asarray(amax, dtype=np.float64)
    _, e = np.frexp(amax)                 # amax = m 2^e, m in [0.5, 1): floor(log2 amax) = e - 1
    X = np.clip(e - 1 - emax, -126, 127)
    return np.where(amax > 0, X, 0)


def round_mx_rows(x, fmt) -> np.ndarray:
    """Every row of x [rows, K] in the MX format: columns [32 b, 32 b + 32) form block b,
    and each block of each row is scaled by its own 2^X and rounded element-wise.
    Returns the values read back."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    for lo in range(0, x.shape[-1], MX_BLOCK):
        v = x[..., lo:lo + MX_BLOCK]
        X = mx_scale_exponent(np.max(np.abs(v), axis=-1, keepdims=True), fmt)
        sc = np.ldexp(1.0, X)
        out[..., lo:lo + MX_BLOCK] = _round_element(v / sc, fmt) * sc
    return out
