"""CPU emulation of the reduced-precision storage formats.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper stores FP32
embeddings (appendix, "Storing Dense Matrix"); BF16 and FP8 storage are
forms added on top of it, so these definitions are readings, not the
paper's:

* BF16: round-to-nearest-even of the FP32 value to 8 significand bits.
* FP8: OCP E4M3FN (4 exponent bits, bias 7, 3 mantissa bits, subnormals,
  largest finite 448, no infinities) with one FP32 scale per row.  The scale
  is ``amax / 448`` (FP32 division); the stored code is the E4M3FN value
  nearest (ties to even) to ``x * (448 / amax)`` (both FP32 operations),
  saturated to +-448.  An all-zero row gets scale 1 and zero codes.

The rounding here is written from the definition of "nearest representable
value": it enumerates the format's value grid and picks the nearest grid
point, resolving exact ties towards the even code.  It is pinned against
PyTorch's own casts in the tests.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP32 -> nearest BF16 (ties to even), returned as FP32 values."""
    x = np.asarray(x, dtype=np.float32)
    x64 = x.astype(np.float64)
    # the two BF16 neighbours of x: truncation towards zero and one step away
    bits = x.view(np.uint32)
    lo_bits = bits & np.uint32(0xFFFF0000)
    lo = lo_bits.view(np.float32).astype(np.float64)
    step = (lo_bits + np.uint32(0x10000)).view(np.float32).astype(np.float64) - lo
    hi = lo + step
    d_lo = np.abs(x64 - lo)
    d_hi = np.abs(hi - x64)
    lo_even = ((lo_bits >> np.uint32(16)) & np.uint32(1)) == 0
    take_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ~lo_even)
    out = np.where(take_hi, hi, lo)
    return out.astype(np.float32)


def _e4m3_grid() -> np.ndarray:
    """All non-negative finite E4M3FN values, indexed by their 7-bit code."""
    vals = []
    for code in range(0x7F):          # 0x7F is NaN
        e, m = code >> 3, code & 7
        if e == 0:
            vals.append(m / 8.0 * 2.0 ** -6)
        else:
            vals.append((1.0 + m / 8.0) * 2.0 ** (e - 7))
    return np.asarray(vals, dtype=np.float64)


E4M3_GRID = _e4m3_grid()
E4M3_MAX = float(E4M3_GRID[-1])      # 448


def e4m3_encode(y: np.ndarray) -> np.ndarray:
    """FP32 values -> E4M3FN codes (uint8), nearest with ties to even code,
    saturating at +-448."""
    y = np.asarray(y, dtype=np.float32).astype(np.float64)
    a = np.minimum(np.abs(y), E4M3_MAX)
    idx = np.searchsorted(E4M3_GRID, a)          # first grid value >= a
    idx = np.clip(idx, 1, len(E4M3_GRID) - 1)
    lo, hi = E4M3_GRID[idx - 1], E4M3_GRID[idx]
    d_lo, d_hi = a - lo, hi - a
    take_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ((idx - 1) % 2 == 1))
    code = np.where(take_hi, idx, idx - 1)
    code = np.where(a == 0, 0, code)
    sign = (y < 0) & (code != 0)
    return (code | (sign.astype(np.int64) << 7)).astype(np.uint8)


def e4m3_decode(code: np.ndarray) -> np.ndarray:
    code = np.asarray(code, dtype=np.uint8)
    v = E4M3_GRID[code & 0x7F]
    return np.where(code & 0x80, -v, v).astype(np.float32)


def fp8_scales(x: np.ndarray) -> np.ndarray:
    """Per-row FP32 scale amax/448 (1 for an all-zero row)."""
    x = np.asarray(x, dtype=np.float32)
    amax = np.abs(x).max(axis=1)
    s = np.where(amax > 0, amax / np.float32(E4M3_MAX), np.float32(1.0))
    return s.astype(np.float32)


def fp8_rows(x: np.ndarray):
    """Quantise rows: returns (dequantised code values as FP32 [n,d], scales
    FP32 [n]); the represented row is values * scale."""
    x = np.asarray(x, dtype=np.float32)
    amax = np.abs(x).max(axis=1).astype(np.float32)
    inv = np.where(amax > 0, np.float32(E4M3_MAX) / np.where(amax > 0, amax, 1),
                   np.float32(1.0)).astype(np.float32)
    y = (x * inv[:, None]).astype(np.float32)
    codes = e4m3_encode(y)
    return e4m3_decode(codes), fp8_scales(x)


def fp8_codes(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    amax = np.abs(x).max(axis=1).astype(np.float32)
    inv = np.where(amax > 0, np.float32(E4M3_MAX) / np.where(amax > 0, amax, 1),
                   np.float32(1.0)).astype(np.float32)
    return e4m3_encode((x * inv[:, None]).astype(np.float32)), fp8_scales(x)
