"""Exact rational evaluation of IEEE single-precision operations (test helper).

Used to pin the oracle's FP32 arithmetic independently of any floating-point unit: every
operation is carried out exactly on Fractions and rounded once to the nearest float32
(ties to even), which is what an IEEE fused multiply-add or division delivers.
"""
from fractions import Fraction

import numpy as np

_EMIN = -126          # smallest normal exponent of binary32
_P = 24               # precision (bits)
_MAXF = (2 - Fraction(1, 2 ** 23)) * Fraction(2) ** 127


def rn32(q: Fraction) -> Fraction:
    """Round a rational to the nearest binary32 value (ties to even); +-inf on overflow."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, _EMIN)
    ulp = Fraction(2) ** (e - (_P - 1))
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    val = fl * ulp
    if val > _MAXF:
        return Fraction(sign) * Fraction(10) ** 60   # stands in for infinity (never hit in tests)
    return sign * val


def f(x) -> Fraction:
    return Fraction(float(np.float32(x)))


def fma(a, b, c) -> Fraction:
    return rn32(f(a) * f(b) + f(c))


def mul(a, b) -> Fraction:
    return rn32(f(a) * f(b))


def div(a, b) -> Fraction:
    return rn32(f(a) / f(b))


def to32(q: Fraction) -> np.float32:
    return np.float32(float(q))
