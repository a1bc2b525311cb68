"""Reference E4M3 rounding for the FP8 storage tests (test infrastructure only).

FP8 storage is not part of the paper (its computations are float64); the
rounding here follows the OCP 8-bit floating point format E4M3: sign bit,
4 exponent bits with bias 7, 3 mantissa bits, subnormals below 2^-6, no
infinities, the all-ones code (S.1111.111) reserved for NaN, so the largest
finite magnitude is 1.75 * 2^8 = 448.  Rounding is to nearest, ties to even,
saturating at 448.  Plain NumPy on float64 values, element by element in
spirit: every finite E4M3 value is listed and the nearest one is chosen.
"""
from __future__ import annotations

import numpy as np

__all__ = ["E4M3_MAX", "e4m3_values", "e4m3_decode", "e4m3_round", "fp8_columns"]

E4M3_MAX = 448.0


def e4m3_decode(code: int) -> float:
    """Value of one 8-bit code."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** -6
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def e4m3_values() -> np.ndarray:
    """The non-negative finite values, ascending (codes 0x00 .. 0x7e)."""
    return np.array([e4m3_decode(c) for c in range(0x7F)])


_POS = e4m3_values()


def e4m3_round(x: np.ndarray) -> np.ndarray:
    """Round each entry to the nearest E4M3 value (ties to the even code,
    i.e. the one whose last mantissa bit is 0), saturating at +-448."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(_POS, a, side="left")          # first value >= a
    hi = np.minimum(hi, len(_POS) - 1)
    lo = np.maximum(hi - 1, 0)
    vlo, vhi = _POS[lo], _POS[hi]
    dlo, dhi = a - vlo, vhi - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    r = np.where(a == vhi, vhi, np.where(pick_hi, vhi, vlo))
    return np.copysign(r, x)


def fp8_columns(P: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per-column scaled E4M3 copy of P: scale_j = max_r |P[r, j]| / 448
    (1 for a zero column) and the value each entry of the copy stands for,
    scale_j * round(P[r, j] / scale_j)."""
    P = np.asarray(P, dtype=np.float64)
    mx = np.max(np.abs(P), axis=0)
    scale = np.where(mx > 0.0, mx / E4M3_MAX, 1.0)
    return e4m3_round(P / scale) * scale, scale
