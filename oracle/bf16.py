"""Reference bfloat16 rounding for the narrow-storage tests (test infrastructure only).

The paper computes in float64 throughout; bfloat16 storage of the factor is
an extension whose rounding is fixed here by the format itself: sign bit,
8 exponent bits with bias 127 (the float32 exponent), 7 stored mantissa
bits, subnormals below 2^-126 with spacing 2^-133, infinities and NaN as in
float32.  A value is rounded ONCE, from float64, to the nearest bfloat16
value with ties to the even significand; magnitudes that round past the
largest finite value (2 - 2^-7) * 2^127 become infinity.

Plain NumPy in float64: the spacing q of the bfloat16 values around |x| is
a power of two, so x / q is exact in float64 and numpy's rint (round half
to even) performs the rounding; the code is the upper half of the float32
bit pattern of the (exactly representable) rounded value.
"""
from __future__ import annotations

import numpy as np

__all__ = ["BF16_MAX", "bf16_round", "bf16_codes", "bf16_decode"]

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Each entry rounded once to the nearest bfloat16 value (ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    out = np.empty_like(x)
    finite = np.isfinite(x)
    nz = finite & (a > 0.0)
    # exponent of the leading bit: a in [2^e, 2^(e+1))
    _, e1 = np.frexp(np.where(nz, a, 1.0))
    e = e1.astype(np.int64) - 1
    q_exp = np.maximum(e, -126) - 7              # spacing 2^q_exp (subnormals: 2^-133)
    r = np.ldexp(np.rint(np.ldexp(np.where(nz, a, 0.0), -q_exp)), q_exp)
    r = np.where(r >= 2.0 ** 128, np.inf, r)     # rounded past the largest finite value
    out[:] = np.where(nz, np.copysign(r, x), x)  # zeros keep their sign; inf/nan pass
    out[~finite] = x[~finite]
    return out


def bf16_codes(x: np.ndarray) -> np.ndarray:
    """The 16-bit codes (uint16) of bf16_round(x); NaN maps to 0x7fc0."""
    r = bf16_round(x)
    codes = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    codes[np.isnan(r)] = 0x7FC0
    return codes


def bf16_decode(codes: np.ndarray) -> np.ndarray:
    """float64 values of 16-bit codes."""
    c = np.asarray(codes, dtype=np.uint32) << 16
    return c.view(np.float32).astype(np.float64)
