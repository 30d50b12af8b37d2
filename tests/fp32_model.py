"""The grid's world -> cell map evaluated in exact rational arithmetic.

The contract's map is a fixed sequence of IEEE-754 binary32 operations,
each rounded to nearest with ties to even:

    ext = RN(hi - lo),  inv = RN(res / ext),  s = RN(p - lo),  u = RN(s * inv),
    cell = min(max(floor(u), 0), res - 1)

This module does every step on Fractions and rounds with ``rn32`` below, which
is written from the definition of the binary32 format (24-bit significand,
exponents down to -126, subnormals at 2^-149, overflow to infinity).  No float
hardware takes part in the arithmetic, so a check of the oracle against this
model does not share the oracle's own rounding.
"""
from fractions import Fraction
import math

_P = 24                       # significand bits, including the implicit one
_EMIN = -126                  # smallest normal exponent
_MAX = (2 - Fraction(1, 2 ** 23)) * Fraction(2) ** 127


def rn32(x: Fraction):
    """x rounded to the nearest binary32 value, ties to the even significand.
    Returns a Fraction, or +-math.inf on overflow."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if a < Fraction(2) ** e:
        e -= 1
    elif a >= Fraction(2) ** (e + 1):
        e += 1
    e = max(e, _EMIN)                      # below the normal range the quantum stays 2^-149
    q = Fraction(2) ** (e - (_P - 1))
    m = a / q
    n = m.numerator // m.denominator       # floor
    r = m - n
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and n % 2 == 1):
        n += 1
    v = n * q
    if v > _MAX:
        return sign * math.inf
    return sign * v


def exact(x) -> Fraction:
    """The exact value of a finite float (a binary32 value converts exactly)."""
    return Fraction(float(x))


def inv_cell(lo, hi, res: int) -> Fraction:
    return rn32(Fraction(int(res)) / rn32(exact(hi) - exact(lo)))


def cell_fp32(p, lo, hi, res: int) -> int:
    """The contract's FP32 map of a finite point p on one axis."""
    inv = inv_cell(lo, hi, res)
    s = rn32(exact(p) - exact(lo))
    u = rn32(s * inv)
    f = math.floor(u)
    return int(min(max(f, 0), int(res) - 1))


def cell_exact(p, lo, hi, res: int) -> int:
    """The same map with no rounding at all (what the FP32 sequence approximates)."""
    u = (exact(p) - exact(lo)) * int(res) / (exact(hi) - exact(lo))
    return int(min(max(math.floor(u), 0), int(res) - 1))
