"""bfloat16 rounding and the hi/lo split used by the split-BF16 products.

bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of an
IEEE-754 binary32 value.  Round-to-nearest-even (the IEEE default rounding)
from binary32: keep the upper 16 bits; if the dropped 16 bits exceed half an
ulp (0x8000) round up, if they equal it round up only when the kept value is
odd; rounding up is +1 on the kept 16-bit integer, which carries into the
exponent (and to infinity) by itself.  NaNs stay NaNs (quiet bit set).

Split of a binary32 value x into two bfloat16 values:
    hi = rne(x),  lo = rne(x - hi)
x - hi is exact in binary32 (hi is x rounded to fewer bits of the same
binade), so hi + lo reproduces x to about 2^-16 relative.
"""
from __future__ import annotations

import numpy as np


def rne_bits(x: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    upper = b >> 16
    rem = b & 0xFFFF
    odd = upper & 1
    round_up = (rem > 0x8000) | ((rem == 0x8000) & (odd == 1))
    out = upper + round_up.astype(np.uint64)
    isnan = np.isnan(x)
    out = np.where(isnan, upper | 0x40, out)
    return (out & 0xFFFF).astype(np.uint16)


def bits_to_float(h: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> binary32 values (exact)."""
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32)


def split(x: np.ndarray):
    """(hi_bits, lo_bits) with hi = rne(x), lo = rne(x - hi), x - hi in binary32."""
    x = np.asarray(x, dtype=np.float32)
    hi = rne_bits(x)
    r = (x - bits_to_float(hi)).astype(np.float32)
    lo = rne_bits(r)
    return hi, lo


def split_value(x: np.ndarray) -> np.ndarray:
    """hi + lo as float64 (the value the split represents)."""
    hi, lo = split(x)
    return bits_to_float(hi).astype(np.float64) + bits_to_float(lo).astype(np.float64)
