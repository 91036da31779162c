"""Exact IEEE-754 binary32/binary64 arithmetic on rationals.

Each operation is computed exactly with ``fractions.Fraction`` and rounded
once, to nearest with ties to even, which is what IEEE-754 defines for
subtraction, multiplication and fused multiply-add.  Tests use it to pin the
oracle's distance routines to the definition of the arithmetic rather than to
another floating-point implementation.  Finite, normal-range values only
(subnormal results are rounded with the fixed minimum exponent).
"""
from fractions import Fraction

import numpy as np


def _round(fr: Fraction, mant_bits: int, emin: int) -> Fraction:
    if fr == 0:
        return Fraction(0)
    sign = -1 if fr < 0 else 1
    a = -fr if fr < 0 else fr
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    scale = Fraction(2) ** (mant_bits - 1 - e)   # ulp = 2^(e - mant_bits + 1)
    m = a * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * Fraction(fl) / scale


def r32(fr: Fraction) -> Fraction:
    return _round(fr, 24, -126)


def r64(fr: Fraction) -> Fraction:
    return _round(fr, 53, -1022)


def F(v) -> Fraction:
    return Fraction(float(v))


def to_f32(fr: Fraction) -> np.float32:
    v = np.float32(float(fr))
    assert Fraction(float(v)) == fr, "value not representable in binary32"
    return v
