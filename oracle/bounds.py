"""Theorem 1 error bounds and the required-moduli reading (test infrastructure only).

est1 is eq. (thm:err-1) of Theorem 1 with the exact |A'B'|; est2 is
eq. (thm:err-2), where |A'B'| is replaced by P/2 (Lemma 0), giving r_b.

  |AB - C_b| <= t |A| v (2^beta')^T + t 2^alpha' v^T |B|
                + (k E + R_b) o t^2 2^alpha' (2^beta')^T,
  t = 1/sqrt(2^5 (P - 1)), alpha' = alpha + e'/2, beta' = beta + f'/2,
  alpha_i = floor(log2 max_h |a_ih|), e'_i = log2 max_h Cbar_ih (likewise beta, f').

Required N (reading R16 of the planner): the paper says the bound tells how
many moduli a desired accuracy needs but fixes no accuracy measure.  The
N-independent part of r_b (the output rounding (3/2) u_64 P, resp.
(1/2) u_32 P) alone exceeds 1e-15 * (|A||B|)_ij, so a target eps is applied to
the N-dependent part

  T_ij(N) = t (|A| v)_i 2^beta'_j + t 2^alpha'_i (v^T |B|)_j
            + (k + r_b(N) - r_b^rnd) t^2 2^alpha'_i 2^beta'_j

relative to S_ij = (|A||B|)_ij: N is the smallest value in [2, 49] with
max_ij T_ij(N) / S_ij <= eps (entries with (|A||B|)_ij = 0 are exact and
skipped; one whose FP64 S_ij underflows to 0 admits no N).
Row and column powers of two are factored out (R18) so nothing overflows.

A-posteriori certification: after a run, Lemma 4 bounds the unknown |A'B'| of
est1 by the computed C'' (|A'B'| <= (|C''| + R_const) / (1 - R_rel)), so est1
itself, output rounding included, can be evaluated from the output; a target
eps is certified when est1_ij <= eps (|A||B|)_ij on every entry with
(|A||B|)_ij > 0, and adaptive N steps N up until it is.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

from .constants import N_MAX, N_MIN, U32, U64, constants
from .ozaki2 import exact_int_matmul, shift_prime, ceil_scaled


def _alpha(maxabs: np.ndarray) -> np.ndarray:
    """floor(log2 max |x|) per row/column (0 for zero rows: never used)."""
    return 5 - shift_prime(maxabs)


def R_const(const) -> Fraction:
    """N-dependent constant part of R_b (Lemma 4), without |A'B'|."""
    N, rho, P = const.N, const.rho, const.P
    if const.b == 64:
        return (1 + 3 * U64) * 2 ** (1 + const.clog2rho) * (N + 2) * U64 ** 2 * rho * P
    return (1 + U32) * (N + 2) * U64 * rho * P


def R_rel(const) -> Fraction:
    """Coefficient of |A'B'| in R_b."""
    return 3 * U64 if const.b == 64 else U32


def _bound_parts(A: np.ndarray, B: np.ndarray, st: dict):
    """The N-dependent pieces of eq. (thm:err-1) per entry, as mpf arrays:
    base = t |A| v (2^beta')^T + t 2^alpha' v^T |B| and tt = t^2 2^alpha' (2^beta')^T,
    plus the constants R_const and R_rel of Lemma 4 and k.  Entries whose row
    or column maximum of Cbar is 0 are exact zeros (R7) and get None."""
    const = st["const"]
    rows, cols = st["rows"], st["cols"]
    k = A.shape[1]
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    alpha = _alpha(A64.max(axis=1))[rows]
    beta = _alpha(B64.max(axis=0))[cols]
    P = mpmath.mpf(const.P)
    t = 1 / mpmath.sqrt(32 * (P - 1))
    Rc = mpmath.mpf(R_const(const).numerator) / R_const(const).denominator
    Rr = mpmath.mpf(R_rel(const).numerator) / R_rel(const).denominator
    rsum = [mpmath.fsum(mpmath.mpf(float(v)) for v in A64[i]) for i in rows]
    csum = [mpmath.fsum(mpmath.mpf(float(v)) for v in B64[:, j]) for j in cols]
    a2 = [mpmath.ldexp(mpmath.sqrt(int(M)), int(al)) for M, al in zip(st["rmax"], alpha)]
    b2 = [mpmath.ldexp(mpmath.sqrt(int(M)), int(be)) for M, be in zip(st["cmax"], beta)]
    base = np.empty((len(rows), len(cols)), dtype=object)
    tt = np.empty((len(rows), len(cols)), dtype=object)
    for x in range(len(rows)):
        for y in range(len(cols)):
            if st["rmax"][x] == 0 or st["cmax"][y] == 0:
                base[x, y] = tt[x, y] = None
                continue
            base[x, y] = t * rsum[x] * b2[y] + t * a2[x] * csum[y]
            tt[x, y] = t * t * a2[x] * b2[y]
    return base, tt, Rc, Rr, P, k


def theorem1(A: np.ndarray, B: np.ndarray, st: dict, ApBp=None):
    """Per-entry est1 (if ApBp, the exact A'B', is given) and est2 as mpf arrays.

    `st` is the stage dict of oracle.ozaki2.os_ii (full or row/col subset).
    """
    with mpmath.workprec(160):
        base, tt, Rc, Rr, P, k = _bound_parts(A, B, st)
        est1 = np.empty(base.shape, dtype=object)
        est2 = np.empty(base.shape, dtype=object)
        for idx in np.ndindex(base.shape):
            if base[idx] is None:
                est1[idx] = est2[idx] = mpmath.mpf(0)   # exact zero output (R7)
                continue
            est2[idx] = base[idx] + (k + Rc + Rr * P / 2) * tt[idx]
            if ApBp is not None:
                est1[idx] = base[idx] + (k + Rc + Rr * abs(int(ApBp[idx]))) * tt[idx]
        return (est1 if ApBp is not None else None), est2


def est1_a_posteriori(A: np.ndarray, B: np.ndarray, st: dict):
    """est1 of eq. (thm:err-1) evaluated after the run, per entry (mpf).

    |A'B'| is not known, but Lemma 4, |A'B' - C''| <= R_const + R_rel |A'B'|,
    bounds it by the computed C'': |A'B'| <= (|C''| + R_const) / (1 - R_rel).
    The result is therefore a bound on |AB - C| that needs only the output
    (and is at least est1 with the exact |A'B'|)."""
    with mpmath.workprec(160):
        base, tt, Rc, Rr, P, k = _bound_parts(A, B, st)
        out = np.empty(base.shape, dtype=object)
        for idx in np.ndindex(base.shape):
            if base[idx] is None:
                out[idx] = mpmath.mpf(0)
                continue
            cpp = abs(mpmath.mpf(float(st["Cpp"][idx])))
            apbp = (cpp + Rc) / (1 - Rr)
            out[idx] = base[idx] + (k + Rc + Rr * apbp) * tt[idx]
        return out


def certified_ratio(A: np.ndarray, B: np.ndarray, st: dict) -> float:
    """max_ij est1_ij / (|A||B|)_ij over the entries of `st` with (|A||B|)_ij > 0
    (a-posteriori est1; exact |A||B|); 0.0 if there is none."""
    from .exact import exact_abs_product
    est = est1_a_posteriori(A, B, st)
    S = exact_abs_product(A, B, st["rows"], st["cols"])
    best = mpmath.mpf(0)
    with mpmath.workprec(160):
        for idx in np.ndindex(est.shape):
            if S[idx] > 0:
                s = mpmath.mpf(S[idx].numerator) / S[idx].denominator
                best = max(best, est[idx] / s)
    return float(best)


def certified_moduli(A: np.ndarray, B: np.ndarray, eps: float, N_start: int, rows=None, cols=None,
                     table: str = "paper"):
    """Adaptive N (a-posteriori certification): starting at N_start, run
    Algorithm 1 and step N up until certified_ratio <= eps.  Returns
    (N, certified, ratio at N); N = the largest admissible N when the target
    is never certified.  With rows/cols the check covers only those entries."""
    from .ozaki2 import os_ii
    b = 64 if A.dtype == np.float64 else 32
    nmax = N_MAX if b == 64 else 16
    ratio = None
    for N in range(max(N_start, N_MIN), nmax + 1):
        _, st = os_ii(A, B, N, rows=rows, cols=cols, stages=True, table=table)
        ratio = certified_ratio(A, B, st)
        if ratio <= eps:
            return N, True, ratio
    return nmax, False, ratio


def planner_terms(A: np.ndarray, B: np.ndarray):
    """N-independent ingredients of T(N) and S in factored form (R18)."""
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    m, k = A64.shape
    n = B64.shape[1]
    amax, bmax = A64.max(axis=1), B64.max(axis=0)
    mu_p, nu_p = shift_prime(amax), shift_prime(bmax)
    Abar = ceil_scaled(A64, mu_p[:, None])
    Bbar = ceil_scaled(B64, nu_p[None, :])
    Cbar = exact_int_matmul(Abar, Bbar, 64.0 * 64.0 * max(k, 1))
    rmax, cmax = Cbar.max(axis=1), Cbar.max(axis=0)
    alpha, beta = 5 - mu_p, 5 - nu_p
    As = np.ldexp(A64, -alpha[:, None].astype(np.int32))         # |A| 2^-alpha, in [0, 2)
    Bs = np.ldexp(B64, -beta[None, :].astype(np.int32))
    # (|A||B|)_ij > 0 exactly when some h has a_ih != 0 and b_hj != 0; the
    # FP64 S below can underflow to 0 for such an entry (a row spanning
    # many binades), and then no N can be certified for it.
    nz = exact_int_matmul((A64 != 0).astype(np.int64), (B64 != 0).astype(np.int64),
                          float(max(k, 1))) > 0
    return dict(k=k, rs=As.sum(axis=1), cs=Bs.sum(axis=0),
                sr=np.sqrt(rmax.astype(np.float64)), sc=np.sqrt(cmax.astype(np.float64)),
                S=As @ Bs, nz=nz)


def ratio_max(terms: dict, N: int, b: int, table: str = "paper") -> tuple:
    """(max_ij T_ij(N)/S_ij, max_ij est2_ij/S_ij) over the entries with
    (|A||B|)_ij > 0; inf when such an entry has an FP64 S_ij of 0."""
    const = constants(N, b, table)
    t = float(1 / mpmath.sqrt(32 * (mpmath.mpf(const.P) - 1)))
    tt_coef = float(Fraction(1, 32 * (const.P - 1)))             # t^2
    extra = float(R_const(const) / (32 * (const.P - 1)))         # (r_b - r_rnd) t^2
    rnd = float(R_rel(const) * Fraction(const.P, 2) / (32 * (const.P - 1)))  # r_rnd t^2
    sr, sc, S = terms["sr"], terms["sc"], terms["S"]
    base = t * (terms["rs"][:, None] * sc[None, :] + sr[:, None] * terms["cs"][None, :])
    prod = sr[:, None] * sc[None, :]
    T = base + (terms["k"] * tt_coef + extra) * prod
    if np.any(terms["nz"] & ~((S > 0) & (prod > 0))):
        return float("inf"), float("inf")
    mask = terms["nz"]
    if not mask.any():
        return 0.0, 0.0
    r1 = float(np.max(T[mask] / S[mask]))
    r2 = float(np.max((T[mask] + rnd * prod[mask]) / S[mask]))
    return r1, r2


def required_moduli_from_terms(terms: dict, eps: float, b: int = 64, table: str = "paper"):
    """Smallest N in [2, 49] (FP32: [2, 16]) whose N-dependent bound is <= eps
    relative to |A||B| on every entry (R16).  Returns (N, reachable, detail)."""
    nmax = N_MAX if b == 64 else 16
    r1 = r2 = None
    for N in range(N_MIN, nmax + 1):
        r1, r2 = ratio_max(terms, N, b, table)
        if r1 <= eps:
            return N, True, dict(ratio=r1, est2_ratio=r2)
    return nmax, False, dict(ratio=r1, est2_ratio=r2)


def required_moduli(A: np.ndarray, B: np.ndarray, eps: float, table: str = "paper"):
    """required_moduli_from_terms(planner_terms(A, B), eps, b, table)."""
    b = 64 if A.dtype == np.float64 else 32
    return required_moduli_from_terms(planner_terms(A, B), eps, b, table)
