"""Complex matrix multiplication by the Ozaki-II scheme (reading R23).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sections 1.1 and 7 name complex GEMM emulation ([uchino_ozaki2_complex]) and
leave its error analysis to future work.  The reading used here applies the
real method, unchanged, to the real embedding of the complex product:

    A = Ar + i Ai (m x k),  B = Br + i Bi (k x n),
    Ahat = [[Ar, -Ai],        Bhat = [[Br],
            [Ai,  Ar]]  (2m x 2k)       [Bi]]  (2k x n),

    Ahat Bhat = [[Ar Br - Ai Bi],  = [[Re AB],
                 [Ai Br + Ar Bi]]     [Im AB]].

So C = os_ii(Ahat, Bhat, N) gives Re C in rows 1..m and Im C in rows
m+1..2m, every quantity of Algorithms 1-3 is the real one for (Ahat, Bhat)
(each output row -- real or imaginary part of a row of C -- gets its own
shift mu, each column its nu), and Lemmas 0-4 and Theorem 1 hold for it with
inner dimension 2k.  The real method's inner-dimension limit therefore
applies to 2k.  The matrix-engine work is four real products of the complex
sizes per modulus (the "4M" form).
"""
from __future__ import annotations

import numpy as np

from .ozaki2 import os_ii


def real_embedding(A: np.ndarray, B: np.ndarray):
    """(Ahat, Bhat) of the module docstring, in the real dtype of A and B."""
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shapes must be (m,k) and (k,n)")
    if A.dtype != B.dtype or A.dtype not in (np.complex128, np.complex64):
        raise ValueError("A and B must both be complex128 or both complex64")
    Ar, Ai = A.real.copy(), A.imag.copy()
    Br, Bi = B.real.copy(), B.imag.copy()
    Ahat = np.block([[Ar, -Ai], [Ai, Ar]])
    Bhat = np.vstack([Br, Bi])
    return Ahat, Bhat


def os_ii_complex(A: np.ndarray, B: np.ndarray, N: int, rows=None, cols=None,
                  stages: bool = False, table: str = "paper"):
    """Complex C (len(rows) x len(cols)) := the real Algorithm 1 on the real
    embedding, reassembled as Re + i Im.  With stages=True also returns the
    real run's stage dictionary (rows of Ahat: the requested rows, then the
    same rows shifted by m)."""
    m = A.shape[0]
    Ahat, Bhat = real_embedding(A, B)
    rows = np.arange(m) if rows is None else np.asarray(rows)
    hrows = np.concatenate([rows, rows + m])
    out = os_ii(Ahat, Bhat, N, rows=hrows, cols=cols, stages=stages, table=table)
    Chat, st = out if stages else (out, None)
    r = len(rows)
    C = Chat[:r] + 1j * Chat[r:]
    C = C.astype(A.dtype)
    return (C, st) if stages else C
