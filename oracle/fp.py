"""Exact IEEE-754 rounding helpers for the oracle (test infrastructure only).

All values are handled as ``fractions.Fraction`` (exact dyadic or general
rationals) and rounded once, the way the paper's notation defines
``fl``, ``fl_down``, ``single``, ``single_down``, ``single_up`` and
``double`` (Section 1.2, "Notation").

Python's ``int / int`` true division is correctly rounded to nearest-even,
so ``float(Fraction)`` is the FP64 round-to-nearest of an exact rational.
"""
from __future__ import annotations

import math
from fractions import Fraction

F32_MANT = 24          # significand bits of FP32 (u_32 = 2^-24)
F32_EMIN = -126        # smallest normal exponent of FP32
F32_EMAX = 127


def floor_log2(x: Fraction) -> int:
    """Exact floor(log2 |x|) of a nonzero rational."""
    x = abs(Fraction(x))
    if x == 0:
        raise ValueError("floor_log2(0)")
    e = x.numerator.bit_length() - x.denominator.bit_length()
    # now 2^(e-1) < x < 2^(e+1); fix up so that 2^e <= x < 2^(e+1)
    if x < Fraction(2) ** e:
        e -= 1
    return e


def round_f32(x, mode: str) -> Fraction:
    """Round a rational to an FP32 value (normal range only).

    mode 'rn' = round to nearest, ties to even (single)
         'rd' = round toward -inf            (single_down / fl_down)
         'ru' = round toward +inf            (single_up)
    """
    x = Fraction(x)
    if x == 0:
        return Fraction(0)
    e = floor_log2(x)
    if not (F32_EMIN <= e <= F32_EMAX):
        raise OverflowError(f"round_f32: exponent {e} outside the FP32 normal range")
    scale = Fraction(2) ** (e - (F32_MANT - 1))     # one unit in the last place
    y = x / scale                                    # |y| in [2^23, 2^24)
    if mode == "rd":
        k = math.floor(y)
    elif mode == "ru":
        k = math.ceil(y)
    elif mode == "rn":
        k = math.floor(y)
        rem = y - k
        if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and k % 2 == 1):
            k += 1
    else:
        raise ValueError(mode)
    return k * scale


def is_f32(x: Fraction) -> bool:
    return round_f32(x, "rn") == Fraction(x)


def rn64(x) -> float:
    """double(x): FP64 round-to-nearest-even of an exact rational."""
    return float(Fraction(x))


def fma64(a: float, b: float, c: float) -> float:
    """fl(fma(a, b, c)): a*b + c computed exactly, rounded once to FP64."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mul64(a: float, b: float) -> float:
    """fl(a * b), one rounding."""
    return float(Fraction(a) * Fraction(b))


def add64(a: float, b: float) -> float:
    """fl(a + b), one rounding."""
    return float(Fraction(a) + Fraction(b))


def ldexp64(x: float, e: int) -> float:
    """fl(x * 2^e) with one rounding (exact unless the result is subnormal)."""
    return float(Fraction(x) * Fraction(2) ** e)
