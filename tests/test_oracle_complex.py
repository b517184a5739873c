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


# --------------------------------------------------------------------------
# The 3-product form (reading R25)
# --------------------------------------------------------------------------
from fractions import Fraction  # noqa: E402

from oracle.bounds import R_const, R_rel  # noqa: E402


def _ints(X):
    return np.vectorize(int, otypes=[object])(X)


def check_3m(A, B, N, table="paper"):
    """Pins of the 3-product form; returns failure strings."""
    bad = []
    C, st = cg.os_ii_complex_3m(A, B, N, stages=True, table=table)
    const = st["const"]
    Ar, Ai = A.real.astype(np.float64), A.imag.astype(np.float64)
    Br, Bi = B.real.astype(np.float64), B.imag.astype(np.float64)
    m, k = A.shape
    n = B.shape[1]
    # Scaling: 2^mu' max(|ar|, |ai|) in [16, 32); Abar = sum of the two
    # ceilings, in [0, 64], and Abar >= 2^mu' (|ar| + |ai|); A' by brute force.
    for i in range(m):
        mx = max(np.abs(Ar[i]).max(), np.abs(Ai[i]).max())
        if mx and not (16 <= Fraction(float(mx)) * Fraction(2) ** int(st["mu_p"][i]) < 32):
            bad.append(f"2^mu' max out of [16, 32) at row {i}")
        for h in range(k):
            s = Fraction(2) ** int(st["mu_p"][i])
            lo = (abs(Fraction(float(Ar[i, h]))) + abs(Fraction(float(Ai[i, h])))) * s
            if not (lo <= int(st["Abar"][i, h]) <= 64):
                bad.append(f"Abar bound at ({i},{h})")
            for X, Xp in ((Ar, st["Apr"]), (Ai, st["Api"])):
                if int(Fraction(float(X[i, h])) * Fraction(2) ** int(st["mu"][i])) != Xp[i, h]:
                    bad.append(f"A' != trunc(2^mu a) at ({i},{h})")
    # Lemma 0 for both parts: (|A'r| + |A'i|)(|B'r| + |B'i|) <= (P - 1) 2^(-1 - 2^-20)
    Aabs = np.abs(st["Apr"]) + np.abs(st["Api"])
    Babs = np.abs(st["Bpr"]) + np.abs(st["Bpi"])
    import mpmath
    with mpmath.workprec(200):
        lim = (mpmath.mpf(const.P) - 1) * mpmath.power(2, -1 - mpmath.mpf(2) ** -20)
        if max((mpmath.mpf(int(v)) for v in Aabs.dot(Babs).reshape(-1)), default=0) > lim:
            bad.append("Lemma 0 bound violated")
    # CRT: W_re, W_im congruent to Re, Im of A'B'; the integer CRT recovers them.
    Re = st["Apr"].dot(st["Bpr"]) - st["Api"].dot(st["Bpi"])
    Im = st["Apr"].dot(st["Bpi"]) + st["Api"].dot(st["Bpr"])
    P = const.P
    red = np.vectorize(lambda v: ((v + P // 2) % P) - P // 2 if P % 2 == 0
                       else ((v + (P - 1) // 2) % P) - (P - 1) // 2, otypes=[object])
    for name, W, T in (("re", st["Wre"], Re), ("im", st["Wim"], Im)):
        acc = np.zeros(T.shape, dtype=object)
        for l, p in enumerate(const.p):
            if np.any(np.mod(W[l].astype(object) - T, p) != 0):
                bad.append(f"W_{name} != {name}(A'B') mod {p}")
            acc = acc + W[l].astype(object) * const.x[l]
        if np.any(red(acc) != T):
            bad.append(f"integer CRT of W_{name} != {name}(A'B')")
    # Lemma 4 per part, and the error of each part of C against the exact
    # product within est = 2 2^-nu rs + 2 2^-mu cs + (4k + R_b) 2^-(mu+nu), with
    # rs_i = sum_h |ar_ih| + |ai_ih|, cs_j = sum_h |br_hj| + |bi_hj| (every
    # truncation error of A', B' below 1 per part).
    re_ex, im_ex = exact_complex(A, B)
    Rc, Rr = R_const(const), R_rel(const)
    for name, T, Cpp, got, ex in (("re", Re, st["Cpp_re"], C.real, re_ex),
                                  ("im", Im, st["Cpp_im"], C.imag, im_ex)):
        for i in range(m):
            rs = sum(abs(Fraction(float(Ar[i, h]))) + abs(Fraction(float(Ai[i, h]))) for h in range(k))
            for j in range(n):
                t = int(T[i, j])
                if abs(t - Fraction(float(Cpp[i, j]))) > Rc + Rr * abs(t):
                    bad.append(f"Lemma 4 ({name}) at ({i},{j})")
                cs = sum(abs(Fraction(float(Br[h, j]))) + abs(Fraction(float(Bi[h, j]))) for h in range(k))
                e = Fraction(2) ** int(-st["mu"][i] - st["nu"][j])
                est = (2 * rs * Fraction(2) ** int(-st["nu"][j]) + 2 * cs * Fraction(2) ** int(-st["mu"][i])
                       + (4 * k + Rc + Rr * abs(t)) * e)
                if abs(Fraction(float(got[i, j])) - ex[i, j]) > est:
                    bad.append(f"error bound ({name}) at ({i},{j})")
    return bad


@pytest.mark.parametrize("N,dt", [(2, np.complex128), (9, np.complex128), (14, np.complex128),
                                  (20, np.complex128), (49, np.complex128), (7, np.complex64),
                                  (16, np.complex64)])
def test_3m_pins(N, dt):
    A, B = complex_gemm_inputs(5, 4, 6, phi=1.0, seed=70 + N, dtype=dt)
    assert check_3m(A, B, N) == []


def test_3m_wide_exponents_zero_rows_optimal_table():
    A, B = complex_gemm_inputs(6, 5, 9, phi=3.0, seed=5)
    A[2, :] = 0
    B[:, 1] = 1e-300 + 0j
    assert check_3m(A, B, 16) == []
    assert check_3m(A, B, 20, table="optimal") == []


def test_3m_int32_wrap_at_the_limit():
    # every residue mod 256 of A'r, A'i, B'r, B'i equal to -128 (N = 14): each
    # p = 256 product sums k terms of 2^14; at k = 2^17 - the largest k whose
    # three products stay one INT32 chunk - they wrap, and the pins still hold.
    from workload import wrap_inputs
    Ar, Br = wrap_inputs(2, 2, 2 ** 17, seed=1)
    Ai, Bi = wrap_inputs(2, 2, 2 ** 17, seed=2)
    _, st = cg.os_ii_complex_3m(Ar + 1j * Ai, Br + 1j * Bi, 14, stages=True)
    assert check_3m(Ar[:, :8] + 1j * Ai[:, :8], Br[:8] + 1j * Bi[:8], 14) == []
    l = list(st["const"].p).index(256)
    P = st["const"].P
    Re = st["Apr"].dot(st["Bpr"]) - st["Api"].dot(st["Bpi"])
    assert np.all(np.mod(st["Wre"][l].astype(object) - Re, 256) == 0)


@pytest.mark.parametrize("mistake", ["im_sign", "sum_sign", "mu_prime"])
def test_3m_planted_mistake_is_caught(monkeypatch, mistake):
    import oracle.ozaki2 as oz2
    if mistake == "mu_prime":
        # the real mu' (one higher): a part's bar can reach 64 and the sum 128
        real_frexp = np.frexp
        monkeypatch.setattr(np, "frexp", lambda x: (real_frexp(x)[0], real_frexp(x)[1] + 1))
        A, B = complex_gemm_inputs(4, 3, 5, phi=1.0, seed=3)
        try:
            bad = check_3m(A, B, 14)
        except AssertionError:
            return
        assert bad != []
        return
    real = cg.residue_products_3m

    def wrong(st):
        out = real(st)
        if mistake == "im_sign":      # W_im = mod(T3 - T1 + T2): T2 counted with the wrong sign
            out["Wim"] = [oz2.mod_sym(w + 2 * oz2.mod_sym(
                oz2.exact_int_matmul(oz2.mod_sym(st["Api"], p), oz2.mod_sym(st["Bpi"], p), 2.0 ** 40), p), p)
                for w, p in zip(out["Wim"], st["const"].p)]
        else:                         # W_re = mod(T1 + T2)
            out["Wre"] = [oz2.mod_sym(w + 2 * oz2.mod_sym(
                oz2.exact_int_matmul(oz2.mod_sym(st["Api"], p), oz2.mod_sym(st["Bpi"], p), 2.0 ** 40), p), p)
                for w, p in zip(out["Wre"], st["const"].p)]
        return out
    monkeypatch.setattr(cg, "residue_products_3m", wrong)
    A, B = complex_gemm_inputs(4, 3, 5, phi=1.0, seed=3)
    assert check_3m(A, B, 14) != []


def test_3m_sampled_rows_and_cols_match_full():
    A, B = complex_gemm_inputs(9, 7, 11, phi=1.0, seed=19)
    full = cg.os_ii_complex_3m(A, B, 13)
    rows, cols = np.array([0, 4, 8]), np.array([2, 6])
    got = cg.os_ii_complex_3m(A, B, 13, rows=rows, cols=cols)
    assert np.array_equal(got, full[np.ix_(rows, cols)])
