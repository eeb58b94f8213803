"""Rounding to the OCP FP8 e4m3 format, in FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The FP8 mode of the library factors the kernel matrix of the points with every
coordinate rounded to e4m3; the oracle of that mode is the FP64 method run on
``round_e4m3(X)``.  The format (OCP 8-bit floating point, E4M3 variant): sign,
4 exponent bits with bias 7, 3 fraction bits; normal values (1 + f/8) 2^e for
e = -6..8 except the all-ones pattern (NaN), so the largest finite value is
1.75 * 2^8 = 448; subnormal values f/8 * 2^-6 (steps of 2^-9).  The reading
used here: round to nearest, ties to an even fraction, and saturate to +-448
beyond the largest finite value; non-finite inputs are returned unchanged.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0
E4M3_MIN_NORMAL_EXP = -6
E4M3_FRACTION_BITS = 3


def round_e4m3(x) -> np.ndarray:
    """Nearest e4m3 value of each element (ties to even, saturating)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    # binade of a: a = m 2^e with m in [0.5, 1), so a lies in [2^(e-1), 2^e)
    _, e = np.frexp(a)
    binade = np.maximum(e.astype(np.int64) - 1, E4M3_MIN_NORMAL_EXP)
    spacing = np.ldexp(1.0, binade - E4M3_FRACTION_BITS)
    q = np.rint(a / spacing) * spacing          # np.rint rounds halves to even
    q = np.where(a >= E4M3_MAX, E4M3_MAX, q)
    out = np.copysign(q, x)
    return np.where(np.isfinite(x), out, x)
