"""Exact reference products for the oracle's checks (test infrastructure only).

AB is formed with exact integer arithmetic: every FP64 entry is m * 2^e with
an integer m, so after scaling each matrix by a power of two every entry is an
integer and the product is an exact big-integer dot product.  The integer
scaling is the measurement helper of workload/reference.py (it holds no step
of the method), shared with the benchmark's error samples.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from workload.reference import int_scaled as _int_scaled


def exact_product(A: np.ndarray, B: np.ndarray, rows=None, cols=None):
    """Exact (AB)[rows][:, cols] as an object array of Fractions."""
    if rows is not None:
        A = A[np.asarray(rows)]
    if cols is not None:
        B = B[:, np.asarray(cols)]
    IA, EA = _int_scaled(A)
    IB, EB = _int_scaled(B)
    P = IA.dot(IB)
    scale = Fraction(2) ** (EA + EB)
    out = np.empty(P.shape, dtype=object)
    for idx in np.ndindex(P.shape):
        out[idx] = P[idx] * scale
    return out


def exact_abs_product(A: np.ndarray, B: np.ndarray, rows=None, cols=None):
    return exact_product(np.abs(A), np.abs(B), rows, cols)


def exact_int_product(Ap: np.ndarray, Bp: np.ndarray) -> np.ndarray:
    """A'B' for object arrays of Python ints (exact, any magnitude)."""
    return Ap.dot(Bp)


def abs_error(C: np.ndarray, AB) -> np.ndarray:
    """|AB - C| entrywise as floats (exact difference, rounded once)."""
    out = np.empty(C.shape, dtype=np.float64)
    for idx in np.ndindex(C.shape):
        out[idx] = float(abs(AB[idx] - Fraction(float(C[idx]))))
    return out
