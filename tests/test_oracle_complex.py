"""Pins of the complex oracle (reading R23: the real method on the real
embedding [[Ar, -Ai], [Ai, Ar]] [[Br], [Bi]]).

- The embedding itself: the exact product of the embedded matrices equals
  the exact complex product's real and imaginary parts (checked with exact
  rational arithmetic, independent of the embedding code's sign and block
  placement).
- Every real pin (Lemmas 0-4, the CRT identity, Theorem 1 against the exact
  product) on the embedded run, and Theorem 1 read back as a bound on the
  complex result's real and imaginary parts.
- Special case: purely real inputs reduce exactly to the real method (the
  zero blocks change no shift), with an exactly zero imaginary part.
- Planted mistakes in the embedding are caught.
"""
import numpy as np
import pytest

import oracle.complex_gemm as cg
from oracle.bounds import theorem1
from oracle.exact import abs_error, exact_product
from oracle.ozaki2 import os_ii
from pins import all_pins
from workload import complex_gemm_inputs

import mpmath


def exact_complex(A, B):
    """(Re AB, Im AB) exactly, as object arrays of Fractions."""
    Ar, Ai = A.real.astype(np.float64), A.imag.astype(np.float64)
    Br, Bi = B.real.astype(np.float64), B.imag.astype(np.float64)
    re = exact_product(Ar, Br) - exact_product(Ai, Bi)
    im = exact_product(Ai, Br) + exact_product(Ar, Bi)
    return re, im


def check_complex(A, B, N):
    m = A.shape[0]
    C, st = cg.os_ii_complex(A, B, N, stages=True)
    Ahat, Bhat = cg.real_embedding(A, B)
    bad = []
    re, im = exact_complex(A, B)
    E = exact_product(Ahat.astype(np.float64), Bhat.astype(np.float64))
    if not (np.array_equal(E[:m], re) and np.array_equal(E[m:], im)):
        bad.append("embedding: exact product of the embedded matrices != exact complex product")
    bad += all_pins(Ahat, Bhat, st)
    est1, _ = theorem1(Ahat, Bhat, st, st["Ap"].dot(st["Bp"]))
    for part, ref, sl in (("re", re, slice(0, m)), ("im", im, slice(m, 2 * m))):
        got = (C.real if part == "re" else C.imag).astype(np.float64)
        err = abs_error(got, ref)
        for idx in np.ndindex(err.shape):
            if mpmath.mpf(err[idx]) > est1[sl][idx]:
                bad.append(f"Theorem 1 violated for the {part} part at {idx}")
                break
    return bad


@pytest.mark.parametrize("N", [2, 7, 14, 20, 33, 49])
def test_complex_pins_fp64(N):
    A, B = complex_gemm_inputs(5, 4, 6, phi=1.0, seed=N)
    assert check_complex(A, B, N) == []


@pytest.mark.parametrize("N", [3, 7, 16])
def test_complex_pins_fp32(N):
    A, B = complex_gemm_inputs(4, 5, 7, phi=0.5, seed=40 + N, dtype=np.complex64)
    assert check_complex(A, B, N) == []


def test_complex_wide_exponents():
    A, B = complex_gemm_inputs(6, 5, 30, phi=4.0, seed=3)
    assert check_complex(A, B, 20) == []


def test_real_inputs_reduce_to_the_real_method():
    from workload import gemm_inputs
    for N, dt, cdt in ((14, np.float64, np.complex128), (7, np.float32, np.complex64)):
        Ar, Br = gemm_inputs(9, 7, 13, phi=1.0, seed=N, dtype=dt)
        C = cg.os_ii_complex(Ar.astype(cdt), Br.astype(cdt), N)
        assert np.array_equal(C.real, os_ii(Ar, Br, N)) and np.all(C.imag == 0)


def test_sampled_rows_and_cols_match_full():
    A, B = complex_gemm_inputs(8, 6, 10, phi=1.0, seed=9)
    full = cg.os_ii_complex(A, B, 12)
    rows, cols = np.array([1, 6]), np.array([0, 5])
    assert np.array_equal(cg.os_ii_complex(A, B, 12, rows=rows, cols=cols), full[np.ix_(rows, cols)])


@pytest.mark.parametrize("mistake", ["sign", "swap"])
def test_planted_embedding_mistake_is_caught(monkeypatch, mistake):
    def wrong(A, B):
        Ar, Ai, Br, Bi = A.real.copy(), A.imag.copy(), B.real.copy(), B.imag.copy()
        if mistake == "sign":       # [[Ar, Ai], [-Ai, Ar]]
            return np.block([[Ar, Ai], [-Ai, Ar]]), np.vstack([Br, Bi])
        return np.block([[Ar, -Ai], [Ai, Ar]]), np.vstack([Bi, Br])   # B blocks swapped
    monkeypatch.setattr(cg, "real_embedding", wrong)
    A, B = complex_gemm_inputs(4, 3, 5, phi=1.0, seed=2)
    assert check_complex(A, B, 14) != []


def test_complex_rejects_bad_input():
    A, B = complex_gemm_inputs(3, 3, 3, seed=1)
    with pytest.raises(ValueError):
        cg.os_ii_complex(A.real.copy(), B.real.copy(), 10)
    with pytest.raises(ValueError):
        cg.os_ii_complex(A, B.astype(np.complex64), 10)
