"""Exact reference arithmetic for the rounding pins: a correctly rounded
fused multiply-add computed with rational numbers (IEEE 754 round to nearest,
ties to even), independent of any C or GPU fma."""
from fractions import Fraction
import math
import struct


def _round_to_format(q: Fraction, mant_bits: int, emin: int) -> Fraction:
    """Rounds q to the nearest value with `mant_bits` significand bits
    (including the implicit one) and minimum normal exponent emin, ties to even."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    # make 2^e <= a < 2^(e+1)
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    ulp = Fraction(2) ** (e - (mant_bits - 1))
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * fl * ulp


def fma64(x: float, a: float, b: float) -> float:
    q = Fraction(x) * Fraction(a) + Fraction(b)
    r = _round_to_format(q, 53, -1022)
    if r == 0:
        # exact zero: +0 unless both addends are -0 (round to nearest)
        prod_neg = (math.copysign(1, x) * math.copysign(1, a)) < 0
        return -0.0 if (prod_neg and x * a == 0 and math.copysign(1, b) < 0 and b == 0) else 0.0
    return float(r)


def f32(v: float) -> float:
    return struct.unpack("<f", struct.pack("<f", v))[0]


def fma32(x: float, a: float, b: float) -> float:
    q = Fraction(f32(x)) * Fraction(f32(a)) + Fraction(f32(b))
    r = _round_to_format(q, 24, -126)
    if r == 0:
        return 0.0
    out = float(r)  # exact: r has 24 significant bits
    assert f32(out) == out
    return out
