"""Algorithms 1-3 of the paper (accurate-mode Ozaki-II), step by step, on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Matrices are numpy arrays in their logical shape: A is (m, k), B is (k, n);
FP64 inputs give b = 64 (DGEMM emulation), FP32 inputs give b = 32 (SGEMM
emulation).  Every step follows the paper's order and notation:

  Algorithm 2 (Scaling):  P', mu', Abar, nu', Bbar, Cbar = Abar Bbar,
                          Dbar = single_up(Cbar), e, f = log2f(row/col max),
                          mu, nu, A' = trunc(2^mu A), B' = trunc(B 2^nu)
  Algorithm 3 (CRT):      A'_l, B'_l = mod(., p_l), C'_l = A'_l B'_l (INT32),
                          W_l = mod(C'_l, p_l), C'(1), C'(2), Q, C''
  Algorithm 1:            C = fl(diag(2^-mu) C'' diag(2^-nu))

Readings where the paper is silent (R numbers shared with the library's documentation):
  R4  a zero row of A (column of B) gets mu' = 0; its outputs are exact zeros.
  R5  Abar is the ceiling of the exact |a| 2^mu'; it is >= 1 for every a != 0.
  R6  log2f is the correctly rounded (nearest-even) FP32 logarithm; it meets
      the paper's accuracy assumption (eq. assumption:log2).
  R7  a zero row maximum of Cbar is replaced by 1 (so e = 0).
  R8  fl_down(floor(fma(c, e, P'))) is evaluated as floor of the FP32
      round-down of the exact c*e + P', which equals floor(c*e + P').
  R10 mod(x, 256) maps the tie 128 to -128 (the INT8 wrap of Section 3.1).
  R11 C'(2) (and C'(1) for b = 32) is the fma chain
      acc = 0; for l = 1..N: acc = fma(s_l, W_l, acc).
  R13 the inverse scaling is one multiplication by 2^(-mu_i - nu_j); for
      b = 32 the FP32 C'' is scaled exactly and rounded once to FP32.
  R14 non-finite input is outside the domain: the oracle raises.
  R22 k may reach 2^19 - 1 (the paper assumes k <= 2^17): Cbar <= 2^12 k
      stays below 2^31, and beyond 2^17 each residue product is formed in
      chunks of 2^17 of k whose residues are added mod p_l (see
      oracle/constants.py, K_MAX_EXT).
  b=32 requires N <= 16 so that the FP32 value single(C'') cannot overflow
      (|A'B'| < P/2 and P/2 < 2^128 only up to N = 16).

Exactness arguments used for speed (each one asserted at run time):
  * Abar Bbar, and A'_l B'_l, are computed with FP64 BLAS: all terms and
    partial sums are integers below 2^53 (entries <= 64 resp. <= 128 in
    magnitude, k < 2^19), so every blocking order gives the exact result
    (eq. 2^29 of Section 3.2 and the bound in Section 3.3).
  * A' = trunc(ldexp(A, mu)) in FP64 is exact: ldexp only rounds when the
    result is below 2^-1022, where trunc gives 0 either way.
  * For b = 64, C'(1) = sum_l s_l1 W_l is exact (Lemma 2); it is formed as an
    exact integer sum and checked to be an FP64 value.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .constants import K_MAX, K_MAX_EXT, constants
from .fp import fma64, ldexp64, mul64, add64, round_f32

# --------------------------------------------------------------------------
# small exact helpers
# --------------------------------------------------------------------------


def _check_inputs(A: np.ndarray, B: np.ndarray) -> int:
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shapes must be (m,k) and (k,n)")
    if A.dtype != B.dtype or A.dtype not in (np.float64, np.float32):
        raise ValueError("A and B must both be float64 or both float32")
    if A.shape[1] > K_MAX_EXT:
        raise ValueError("k must be below 2^19 (Section 3's k <= 2^17, widened by reading R22)")
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(B))):
        raise ValueError("non-finite input is outside the domain of the method (R14)")
    return 64 if A.dtype == np.float64 else 32


def shift_prime(maxabs: np.ndarray) -> np.ndarray:
    """mu'_i = 5 - floor(log2 max_h |a_ih|)  (Algorithm 2; eq. mu'nu').

    np.frexp is exact (also for subnormals): x = f 2^e with f in [0.5, 1),
    so floor(log2 x) = e - 1.  Zero maxima get 0 (R4).
    """
    _, e = np.frexp(maxabs.astype(np.float64))
    out = 6 - e.astype(np.int64)
    out[maxabs == 0] = 0
    return out


def ceil_scaled(absX: np.ndarray, shift: np.ndarray) -> np.ndarray:
    """Abar = ceil(2^mu' |A|) as int64 (R5: >= 1 where the entry is nonzero)."""
    v = np.ceil(np.ldexp(absX, shift.astype(np.int32)))
    v = np.where(absX != 0, np.maximum(v, 1.0), 0.0)
    assert v.size == 0 or (v.min() >= 0 and v.max() <= 64), "Abar must lie in [0, 64] (Section 3.2)"
    return v.astype(np.int64)


def single_up_int(M: int) -> int:
    """single_up of a nonnegative integer (exact below 2^24)."""
    return int(round_f32(Fraction(M), "ru")) if M > 0 else 0


_LOG2F_CACHE: dict = {}


def log2f(d: int) -> Fraction:
    """R6: correctly rounded FP32 log2 of an integer-valued FP32 number d >= 1."""
    if d in _LOG2F_CACHE:
        return _LOG2F_CACHE[d]
    if d & (d - 1) == 0:                      # power of two: exact
        r = Fraction(d.bit_length() - 1)
    else:
        import mpmath
        from .constants import mpf_to_fraction
        with mpmath.workprec(200):
            v = mpf_to_fraction(mpmath.log(mpmath.mpf(d), 2))
        r = round_f32(v, "rn")
        # log2 of a non-power-of-two integer is irrational; make sure the
        # 200-bit value is far from an FP32 rounding boundary.
        ulp = Fraction(2) ** (math.floor(math.log2(float(r))) - 23 if r != 0 else -149)
        mid_lo, mid_hi = r - ulp / 2, r + ulp / 2
        assert min(abs(v - mid_lo), abs(v - mid_hi)) > Fraction(1, 2 ** 180)
    _LOG2F_CACHE[d] = r
    return r


def shift(mu_prime: int, cmax: int, const) -> int:
    """mu_i = mu'_i + fl_down(floor(fma(c, e_i, P')))  (Algorithm 2)."""
    d = single_up_int(max(int(cmax), 1))      # Dbar = single_up(Cbar); R7 for zero maxima
    e = log2f(d)
    y = round_f32(const.c * e + const.Pprime, "rd")   # FP32 fma in round-down mode
    return int(mu_prime) + math.floor(y)


def mod_sym(X, p: int) -> np.ndarray:
    """mod(x, p) = x - p round(x/p) stored as INT8 (Section 1.2; R10).

    X may be an object array of Python ints or an integer numpy array.
    """
    r = np.mod(X, p)                          # Python / numpy floor-mod: [0, p)
    r = np.asarray(r).astype(np.int64)
    r[r >= (p + 1) // 2] -= p                 # odd p: (p/2, p) -> negative; p=256: 128 -> -128
    return r


def wrap_int32(X: np.ndarray) -> np.ndarray:
    return ((X + 2 ** 31) % 2 ** 32) - 2 ** 31


def exact_int_matmul(X: np.ndarray, Y: np.ndarray, bound: float) -> np.ndarray:
    """Integer matrix product via FP64 BLAS; exact because |terms| and partial
    sums stay below 2^53 (bound = max |x| * max |y| * k)."""
    assert bound < 2.0 ** 53
    return np.rint(X.astype(np.float64) @ Y.astype(np.float64)).astype(np.int64)


def to_int_objects(V: np.ndarray) -> np.ndarray:
    """FP64 integer values -> object array of exact Python ints."""
    out = np.empty(V.shape, dtype=object)
    flat, src = out.reshape(-1), V.reshape(-1)
    for t in range(src.size):
        flat[t] = int(src[t])
    return out


# --------------------------------------------------------------------------
# Algorithm 2: Scaling
# --------------------------------------------------------------------------


def scaling(A: np.ndarray, B: np.ndarray, N: int, rows=None, cols=None,
            table: str = "paper") -> dict:
    """Algorithm 2.  With `rows`/`cols` given, mu and A' are produced only for
    those rows of A and nu and B' only for those columns of B (the row and
    column maxima of Cbar they need are still taken over the full matrices).
    `table` selects the moduli (oracle.constants.moduli_for)."""
    b = _check_inputs(A, B)
    const = constants(N, b, table)
    m, k = A.shape
    n = B.shape[1]
    rows = np.arange(m) if rows is None else np.asarray(rows)
    cols = np.arange(n) if cols is None else np.asarray(cols)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)          # exact widening
    absA, absB = np.abs(A64), np.abs(B64)

    mu_p = shift_prime(absA.max(axis=1) if k else np.zeros(m))       # mu'
    nu_p = shift_prime(absB.max(axis=0) if k else np.zeros(n))       # nu'
    Abar = ceil_scaled(absA, mu_p[:, None])                           # Abar
    Bbar = ceil_scaled(absB, nu_p[None, :])                           # Bbar

    # Cbar = Abar Bbar on "INT8 matrix engines"; exact integers <= 2^12 k
    # (<= 2^29 for k <= 2^17; below 2^31 for k < 2^19, reading R22).
    bound = 64.0 * 64.0 * max(k, 1)
    full = len(rows) == m and len(cols) == n
    if full:
        Cbar = exact_int_matmul(Abar, Bbar, bound)
        rmax = Cbar.max(axis=1) if n else np.zeros(m, np.int64)
        cmax = Cbar.max(axis=0) if m else np.zeros(n, np.int64)
        rmax, cmax = rmax[rows], cmax[cols]
    else:
        Cbar = None
        rmax = exact_int_matmul(Abar[rows], Bbar, bound).max(axis=1)
        cmax = exact_int_matmul(Abar, Bbar[:, cols], bound).max(axis=0)
    assert rmax.size == 0 or rmax.max() <= 2 ** 12 * k < 2 ** 31

    mu = np.array([shift(mu_p[i], rmax[t], const) for t, i in enumerate(rows)], dtype=np.int64)
    nu = np.array([shift(nu_p[j], cmax[t], const) for t, j in enumerate(cols)], dtype=np.int64)

    # A' = trunc(diag(2^mu) A), B' = trunc(B diag(2^nu)); exact in FP64.
    Ap = np.trunc(np.ldexp(A64[rows, :], mu[:, None].astype(np.int32)))
    Bp = np.trunc(np.ldexp(B64[:, cols], nu[None, :].astype(np.int32)))
    return dict(b=b, const=const, rows=rows, cols=cols, mu_p=mu_p, nu_p=nu_p,
                Abar=Abar, Bbar=Bbar, Cbar=Cbar, rmax=rmax, cmax=cmax, mu=mu, nu=nu,
                Ap=to_int_objects(Ap), Bp=to_int_objects(Bp))


# --------------------------------------------------------------------------
# Algorithm 3: CRT
# --------------------------------------------------------------------------


def residue_products(Ap: np.ndarray, Bp: np.ndarray, const) -> dict:
    """Algorithm 3, residue steps: A'_l, B'_l, C'_l (INT32) and W_l.

    For k <= 2^17, C'_l is the INT32 product (two's complement; it wraps only
    for p = 256, where the wrap keeps it congruent mod 256) and
    W_l = mod(C'_l, p_l).  For larger k (reading R22) the product is formed
    in chunks of 2^17 of k, each such INT32 product, and
    W_l = mod(sum of the chunks' mod(., p_l), p_l); the stage C'_l then
    holds the exact product A'_l B'_l (int64)."""
    k = Ap.shape[1]
    Al, Bl, Cl, W = [], [], [], []
    for p in const.p:
        a = mod_sym(Ap, p)
        bm = mod_sym(Bp, p)
        if k <= K_MAX:
            c = wrap_int32(exact_int_matmul(a, bm, 128.0 * 128.0 * max(k, 1)))
            w = mod_sym(c, p)
        else:
            c = exact_int_matmul(a, bm, 128.0 * 128.0 * k)
            w = np.zeros(c.shape, dtype=np.int64)
            for h0 in range(0, k, K_MAX):
                part = wrap_int32(exact_int_matmul(a[:, h0:h0 + K_MAX], bm[h0:h0 + K_MAX],
                                                   128.0 * 128.0 * K_MAX))
                w = mod_sym(w + mod_sym(part, p), p)
        Al.append(a)
        Bl.append(bm)
        Cl.append(c)
        W.append(w)
    return dict(Al=Al, Bl=Bl, Cl=Cl, W=W)


_fma_v = np.frompyfunc(fma64, 3, 1)
_mul_v = np.frompyfunc(mul64, 2, 1)
_add_v = np.frompyfunc(add64, 2, 1)


def crt_reconstruct(W: list, const) -> dict:
    """Algorithm 3, accumulation and final reduction: C'(1), C'(2), Q, C''."""
    shape = W[0].shape
    Wo = [w.astype(object) for w in W]
    if const.b == 64:
        # C'(1) = fl(sum s_l1 W_l) is exact (Lemma 2): integer sum, checked.
        acc = np.zeros(shape, dtype=object)
        for s, w in zip(const.s1_int, Wo):
            acc = acc + w * s
        C1 = np.empty(shape, dtype=object)
        for idx, v in np.ndenumerate(acc):
            f = float(v)
            assert int(f) == v, "C'(1) must be exactly representable (Lemma 2)"
            C1[idx] = f
        C2 = np.full(shape, 0.0, dtype=object)
        for s, w in zip(const.s2, Wo):                  # R11: fma chain in l order
            C2 = _fma_v(s, w, C2)
    else:
        C1 = np.full(shape, 0.0, dtype=object)
        for s, w in zip(const.s1, Wo):                  # R11 for b = 32
            C1 = _fma_v(s, w, C1)
        C2 = np.full(shape, 0.0, dtype=object)
    # Q = round(fl(P_inv C'(1)));  ties cannot occur (Lemma 3).
    Q = np.frompyfunc(lambda v: float(round(v)), 1, 1)(_mul_v(const.Pinv, C1))
    negQ = np.frompyfunc(lambda v: -v, 1, 1)(Q)
    T = _fma_v(negQ, const.P1, C1)                      # fma(-Q, P1, C'(1))
    if const.b == 64:
        Cpp = _fma_v(negQ, const.P2, _add_v(T, C2))     # fma(-Q, P2, T + C'(2))
    else:
        Cpp = np.frompyfunc(lambda v: float(np.float32(v)), 1, 1)(T)   # single(C'')
    return dict(C1=C1.astype(np.float64), C2=C2.astype(np.float64),
                Q=Q.astype(np.float64), Cpp=Cpp.astype(np.float64))


def unscale(Cpp: np.ndarray, mu: np.ndarray, nu: np.ndarray, b: int) -> np.ndarray:
    """Algorithm 1, last step: C = fl(diag(2^-mu) C'' diag(2^-nu)) (R13)."""
    m, n = Cpp.shape
    out = np.empty((m, n), dtype=np.float64)
    for i in range(m):
        for j in range(n):
            out[i, j] = ldexp64(float(Cpp[i, j]), -int(mu[i]) - int(nu[j]))
    if b == 32:
        # C'' is an FP32 value; the exact scaled value fits FP64, so this is
        # one rounding to FP32.
        return out.astype(np.float32)
    return out


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------


def os_ii(A: np.ndarray, B: np.ndarray, N: int, rows=None, cols=None, stages: bool = False,
          table: str = "paper"):
    """C := OS_II(A, B, p) with p the first N moduli of the list of Section 3.1
    (table="paper") or the per-N moduli of largest product (table="optimal")
    (Algorithm 1).

    Returns C (shape len(rows) x len(cols), FP64 or FP32); with stages=True
    returns (C, dict of every intermediate quantity).
    """
    b = _check_inputs(A, B)
    if b == 32 and N > 16:
        raise ValueError("b = 32 requires N <= 16 (single(C'') must not overflow)")
    m, k = A.shape
    n = B.shape[1]
    nr = m if rows is None else len(rows)
    nc = n if cols is None else len(cols)
    dt = np.float64 if b == 64 else np.float32
    if nr == 0 or nc == 0 or k == 0:
        C = np.zeros((nr, nc), dtype=dt)              # BLAS convention: C = 0
        return (C, {}) if stages else C
    st = scaling(A, B, N, rows, cols, table)
    st.update(residue_products(st["Ap"], st["Bp"], st["const"]))
    st.update(crt_reconstruct(st["W"], st["const"]))
    C = unscale(st["Cpp"], st["mu"], st["nu"], b)
    st["C"] = C
    return (C, st) if stages else C


def log2f_many(d: np.ndarray) -> np.ndarray:
    """R6 (correctly rounded FP32 log2) for many integer-valued FP32 inputs.

    FP64 log2 is within a few ulp of the real value (relative error far below
    2^-40); an FP32 result can only be decided wrongly from it when the FP64
    value lies within 2^-40 (relative) of an FP32 rounding midpoint, and those
    inputs are settled one by one with log2f()."""
    d = np.asarray(d, dtype=np.float32)
    v = np.log2(d.astype(np.float64))
    r = v.astype(np.float32)                              # nearest FP32 of the FP64 value
    rd = r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
    mid_up, mid_dn = 0.5 * (rd + up), 0.5 * (rd + dn)
    tol = np.abs(v) * 2.0 ** -40
    near = (np.abs(v - mid_up) <= tol) | (np.abs(v - mid_dn) <= tol)
    out = r.copy()
    for idx in np.nonzero(near)[0]:
        out[idx] = np.float32(float(log2f(int(d[idx]))))
    return out
