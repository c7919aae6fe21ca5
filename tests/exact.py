"""Exact-arithmetic helpers used to pin the oracle.

Every result here is computed with Python rationals (fractions.Fraction) and
rounded once, correctly, to the target format.  CPython's int/int true
division is correctly rounded, so float(Fraction) is round-to-nearest-even to
binary64; binary32 and bfloat16 rounding are done with integer arithmetic.
"""
from fractions import Fraction

import numpy as np


def fma64(a, b, c):
    """Correctly rounded a*b + c in binary64."""
    return float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def round_binary(q, mant_bits, emin):
    """Round a Fraction to the nearest value with `mant_bits` significand bits
    (including the implicit one) and minimum exponent `emin` (of the leading
    bit), ties to even.  Returns a Fraction.  No overflow handling."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    q = abs(q)
    # exponent of the leading bit: 2^e <= q < 2^(e+1)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    e = max(e, emin)
    scale = Fraction(2) ** (e - (mant_bits - 1))        # weight of the last kept bit
    m = q / scale
    n, r = divmod(m.numerator, m.denominator)
    twice = 2 * r
    if twice > m.denominator or (twice == m.denominator and (n & 1)):
        n += 1
    return sign * n * scale


def to_f32(q):
    """Correctly rounded binary32 value of a Fraction (returned as np.float32)."""
    v = round_binary(Fraction(q), 24, -126)
    return np.float32(float(v))


def fma32(a, b, c):
    return to_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def bf16(x):
    """bfloat16 round-to-nearest-even of a binary32 value (returned as np.float32)."""
    v = round_binary(Fraction(float(np.float32(x))), 8, -126)
    return np.float32(float(v))


def pairwise_recursive(d):
    """The pairwise tree defined recursively: split at the largest power of two
    below n, sum each side the same way, add the two halves."""
    d = [float(x) for x in d]

    def rec(lo, hi):
        n = hi - lo
        if n == 1:
            return d[lo]
        p = 1
        while p * 2 < n:
            p *= 2
        return rec(lo, lo + p) + rec(lo + p, hi)

    if not d:
        return 0.0
    return rec(0, len(d))
