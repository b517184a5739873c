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


# --------------------------------------------------------------------------
# The 3-product form (reading R25)
# --------------------------------------------------------------------------
#
# Three real residue products per modulus instead of four (Gauss's
# identity): with T1 = A'r B'r, T2 = A'i B'i, T3 = (A'r + A'i)(B'r + B'i),
#     Re(A'B') = T1 - T2,   Im(A'B') = T3 - T1 - T2.
# T1, T2 and T3 share one shift per row of A and one per column of B, so
# Algorithm 2 is applied to the complex matrices as wholes:
#   * mu'_i = 4 - floor(log2 max_h max(|ar_ih|, |ai_ih|)) (one lower than the
#     real mu', so that each part's bar is at most 32);
#   * Abar = ceil(2^mu' |Ar|) + ceil(2^mu' |Ai|) in [0, 64] (each term >= 1
#     for a nonzero part, R5), and likewise Bbar; then Cbar = Abar Bbar,
#     Dbar, e, f, mu, nu exactly as in the real Algorithm 2;
#   * A'r = trunc(2^mu Ar), A'i = trunc(2^mu Ai), B'r, B'i likewise.
# Since 2^mu' (|ar| + |ai|) <= Abar, Cbar bounds 2^(mu'+nu') (|Ar|+|Ai|)(|Br|+|Bi|)
# entrywise, and Lemma 0's argument, unchanged, gives
# (|A'r| + |A'i|)(|B'r| + |B'i|) < P/2, which bounds |Re A'B'| and |Im A'B'|:
# the CRT of Algorithm 3 recovers both from
#     W_re = mod(T1 - T2, p_l),   W_im = mod(T3 - T1 - T2, p_l),
# each residue product formed from the INT8 residues mod(A'r, p_l),
# mod(A'i, p_l) and mod(A'r + A'i, p_l) (= mod of the sum of the first two).


def _split(X):
    return X.real.astype(np.float64), X.imag.astype(np.float64)


def scaling_3m(A: np.ndarray, B: np.ndarray, N: int, table: str = "paper", rows=None,
               cols=None) -> dict:
    """Algorithm 2 on complex A, B for the 3-product form (see above).  With
    `rows`/`cols` given, mu and the scaled parts are produced only for those
    rows of A and columns of B (the maxima of Cbar are still taken over the
    full matrices)."""
    from .constants import constants
    from .ozaki2 import exact_int_matmul, shift, to_int_objects

    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shapes must be (m,k) and (k,n)")
    if A.dtype != B.dtype or A.dtype not in (np.complex128, np.complex64):
        raise ValueError("A and B must both be complex128 or both complex64")
    m, k = A.shape
    n = B.shape[1]
    from .constants import K_MAX_EXT
    if k > K_MAX_EXT:
        raise ValueError("k must be below 2^19 (Cbar <= 2^12 k as in the real method)")
    Ar, Ai = _split(A)
    Br, Bi = _split(B)
    if not all(np.all(np.isfinite(X)) for X in (Ar, Ai, Br, Bi)):
        raise ValueError("non-finite input is outside the domain of the method (R14)")
    b = 64 if A.dtype == np.complex128 else 32
    const = constants(N, b, table)

    def mu_prime(mx):
        _, e = np.frexp(mx)
        out = 5 - e.astype(np.int64)               # 4 - floor(log2 mx); frexp exact
        out[mx == 0] = 0                           # R4
        return out

    def bar(X, sh):
        v = np.ceil(np.ldexp(np.abs(X), sh.astype(np.int32)))
        v = np.where(X != 0, np.maximum(v, 1.0), 0.0)
        assert v.size == 0 or v.max() <= 32, "each part's bar lies in [0, 32]"
        return v.astype(np.int64)

    mxA = np.maximum(np.abs(Ar), np.abs(Ai)).max(axis=1) if k else np.zeros(m)
    mxB = np.maximum(np.abs(Br), np.abs(Bi)).max(axis=0) if k else np.zeros(n)
    mu_p, nu_p = mu_prime(mxA), mu_prime(mxB)
    Abar = bar(Ar, mu_p[:, None]) + bar(Ai, mu_p[:, None])
    Bbar = bar(Br, nu_p[None, :]) + bar(Bi, nu_p[None, :])
    bound = 64.0 * 64.0 * max(k, 1)
    if rows is None and cols is None:
        Cbar = exact_int_matmul(Abar, Bbar, bound)
        rmax = Cbar.max(axis=1) if n else np.zeros(m, np.int64)
        cmax = Cbar.max(axis=0) if m else np.zeros(n, np.int64)
        rows, cols = np.arange(m), np.arange(n)
    else:
        rows = np.arange(m) if rows is None else np.asarray(rows)
        cols = np.arange(n) if cols is None else np.asarray(cols)
        rmax = exact_int_matmul(Abar[rows], Bbar, bound).max(axis=1)
        cmax = exact_int_matmul(Abar, Bbar[:, cols], bound).max(axis=0)
    mu = np.array([shift(mu_p[i], rmax[t], const) for t, i in enumerate(rows)], dtype=np.int64)
    nu = np.array([shift(nu_p[j], cmax[t], const) for t, j in enumerate(cols)], dtype=np.int64)
    sc = lambda X, s: to_int_objects(np.trunc(np.ldexp(X, s.astype(np.int32))))
    return dict(b=b, const=const, rows=rows, cols=cols, mu_p=mu_p, nu_p=nu_p, Abar=Abar,
                Bbar=Bbar, rmax=rmax, cmax=cmax, mu=mu, nu=nu,
                Apr=sc(Ar[rows], mu[:, None]), Api=sc(Ai[rows], mu[:, None]),
                Bpr=sc(Br[:, cols], nu[None, :]), Bpi=sc(Bi[:, cols], nu[None, :]))


def residue_products_3m(st: dict) -> dict:
    """The three residue products per modulus and W_re, W_im."""
    from .constants import K_MAX
    from .ozaki2 import exact_int_matmul, mod_sym, wrap_int32

    k = st["Apr"].shape[1]

    def prod(a, b_, p):                      # W of one INT32 residue product (R22 chunks)
        w = np.zeros((a.shape[0], b_.shape[1]), dtype=np.int64)
        for h0 in range(0, max(k, 1), K_MAX):
            part = wrap_int32(exact_int_matmul(a[:, h0:h0 + K_MAX], b_[h0:h0 + K_MAX],
                                               128.0 * 128.0 * K_MAX))
            w = mod_sym(w + mod_sym(part, p), p)
        return w

    Wre, Wim = [], []
    for p in st["const"].p:
        ar, ai = mod_sym(st["Apr"], p), mod_sym(st["Api"], p)
        br, bi = mod_sym(st["Bpr"], p), mod_sym(st["Bpi"], p)
        as_, bs = mod_sym(ar + ai, p), mod_sym(br + bi, p)
        t1, t2, t3 = prod(ar, br, p), prod(ai, bi, p), prod(as_, bs, p)
        Wre.append(mod_sym(t1 - t2, p))
        Wim.append(mod_sym(t3 - t1 - t2, p))
    return dict(Wre=Wre, Wim=Wim)


def os_ii_complex_3m(A: np.ndarray, B: np.ndarray, N: int, stages: bool = False,
                     table: str = "paper", rows=None, cols=None):
    """Complex C (len(rows) x len(cols)) by the 3-product form (reading R25):
    Algorithm 2 as above, three residue products per modulus, the CRT of
    Algorithm 3 on the real and on the imaginary residues, and the inverse
    scaling of Algorithm 1."""
    from .ozaki2 import crt_reconstruct, unscale

    st = scaling_3m(A, B, N, table, rows, cols)
    m, n = len(st["rows"]), len(st["cols"])
    if A.shape[1] == 0 or m == 0 or n == 0:
        C = np.zeros((m, n), dtype=A.dtype)
        return (C, st) if stages else C
    st.update(residue_products_3m(st))
    re = crt_reconstruct(st["Wre"], st["const"])
    im = crt_reconstruct(st["Wim"], st["const"])
    st["Cpp_re"], st["Cpp_im"] = re["Cpp"], im["Cpp"]
    Cr = unscale(re["Cpp"], st["mu"], st["nu"], st["b"])
    Ci = unscale(im["Cpp"], st["mu"], st["nu"], st["b"])
    C = (Cr.astype(np.float64) + 1j * Ci.astype(np.float64)).astype(A.dtype)
    return (C, st) if stages else C
