"""Round-to-nearest-even onto the reduced-precision grids, written from the formats'
definitions (test infrastructure; never on the product path).

The paper names reduced precision ("quantization ... and kernel fusion") as the next
step for its TabNet inference (Sec. VI-D).  The oracle can round GEMM operands the way
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
