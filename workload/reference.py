"""Exact reference values of AB, for error measurement.

Not part of the method (no step of Ozaki-II is here): every FP64 entry is an
integer times a power of two, so after scaling each matrix by one power of
two its entries are integers and AB is an exact big-integer product.  The
benchmark's error samples and the oracle's exact products (oracle/exact.py)
both use int_scaled, so the exact-product code exists once.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def int_scaled(X: np.ndarray):
    """(object array of Python ints I, exponent E) with X == I * 2^E exactly."""
    X = X.astype(np.float64)
    f, e = np.frexp(X)
    mant = np.ldexp(f, 53).astype(np.int64)
    e = e.astype(np.int64) - 53
    nz = mant != 0
    E = int(e[nz].min()) if nz.any() else 0
    out = np.empty(X.shape, dtype=object)
    for idx in np.ndindex(X.shape):
        out[idx] = int(mant[idx]) << int(e[idx] - E) if mant[idx] else 0
    return out, E


class ExactSamples:
    """Exact (AB)_ij and (|A||B|)_ij at the sampled rows x columns."""

    def __init__(self, A: np.ndarray, B: np.ndarray, rows, cols):
        Ar, Bc = A[np.asarray(rows)], B[:, np.asarray(cols)]
        IA, EA = int_scaled(Ar)
        IB, EB = int_scaled(Bc)
        P = IA.dot(IB)
        scale = Fraction(2) ** (EA + EB)
        self.AB = np.empty(P.shape, dtype=object)
        for idx in np.ndindex(P.shape):
            self.AB[idx] = P[idx] * scale
        self.S = np.abs(Ar.astype(np.float64)) @ np.abs(Bc.astype(np.float64))

    def rel_error(self, Csub: np.ndarray) -> float:
        """max |C_ij - (AB)_ij| / (|A||B|)_ij over the samples (Csub holds them)."""
        worst = 0.0
        for idx in np.ndindex(self.AB.shape):
            if self.S[idx] == 0:
                continue
            err = abs(Fraction(float(Csub[idx])) - self.AB[idx])
            worst = max(worst, float(err) / self.S[idx])
        return worst


def sampled_relative_error(A: np.ndarray, B: np.ndarray, C: np.ndarray, rows, cols) -> float:
    """One-shot form of ExactSamples(...).rel_error(C)."""
    return ExactSamples(A, B, rows, cols).rel_error(C)
