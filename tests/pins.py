"""Independent checks ("pins") of the oracle's stages against what the paper
and plain mathematics fix.  Each function returns a list of failure strings
(empty = pass) so that the same checks serve the pin tests and the
planted-mistake tests.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

from oracle.bounds import R_const, R_rel, theorem1
from oracle.constants import U32, U64
from oracle.exact import abs_error, exact_product


def _abs_int(X):
    return np.vectorize(lambda v: abs(int(v)), otypes=[object])(X)


def pin_scaling(A, B, st):
    """Section 3.2 facts: 2^mu' max|a| in [32, 64); Abar, Bbar in [0, 64] and
    Abar >= 2^mu'|A| (a ceiling); Cbar row/col maxima <= 2^12 k (< 2^31); A' equals
    trunc(2^mu a) computed with exact rationals."""
    bad = []
    A64, B64 = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    rows, cols = st["rows"], st["cols"]
    amax = A64.max(axis=1)
    for i in range(A.shape[0]):
        if amax[i] != 0:
            v = Fraction(float(amax[i])) * Fraction(2) ** int(st["mu_p"][i])
            if not (32 <= v < 64):
                bad.append(f"2^mu' max|a| out of [32,64) at row {i}")
    Ab = st["Abar"]
    if Ab.min() < 0 or Ab.max() > 64:
        bad.append("Abar out of [0,64]")
    scaled = np.ldexp(A64, st["mu_p"][:, None].astype(np.int32))
    if np.any(Ab < scaled) or np.any(Ab >= scaled + 1):
        bad.append("Abar is not the ceiling of 2^mu'|A|")
    lim = 2 ** 12 * A.shape[1]                     # eq. (2^29): 2^12 k, <= 2^29 for k <= 2^17
    if st["rmax"].max(initial=0) > lim or st["cmax"].max(initial=0) > lim or lim >= 2 ** 31:
        bad.append("Cbar maximum exceeds 2^12 k, or 2^12 k reaches 2^31")
    for t, i in enumerate(rows):
        for h in range(A.shape[1]):
            ref = int(Fraction(float(A[i, h])) * Fraction(2) ** int(st["mu"][t]))
            if ref != st["Ap"][t, h]:
                bad.append(f"A' != trunc(2^mu a) at ({i},{h})")
                return bad
    for t, j in enumerate(cols):
        for h in range(B.shape[0]):
            ref = int(Fraction(float(B[h, j])) * Fraction(2) ** int(st["nu"][t]))
            if ref != st["Bp"][h, t]:
                bad.append(f"B' != trunc(b 2^nu) at ({h},{j})")
                return bad
    return bad


def pin_lemma0_lemma1(A, B, st):
    """Lemma 0 in its rigorous form |A'||B'| <= (P-1) 2^(-1-2^-20), and the
    Lemma 1 lower bound mu_i >= -alpha'_i + (log2(P-1) + 5)/2."""
    bad = []
    const = st["const"]
    AB = _abs_int(st["Ap"]).dot(_abs_int(st["Bp"]))
    with mpmath.workprec(200):
        lim = (mpmath.mpf(const.P) - 1) * mpmath.power(2, -1 - mpmath.mpf(2) ** -20)
        if max((mpmath.mpf(int(v)) for v in AB.reshape(-1)), default=0) > lim:
            bad.append("Lemma 0 violated: |A'||B'| > (P-1) 2^(-1-2^-20)")
        A64 = np.abs(A.astype(np.float64))
        B64 = np.abs(B.astype(np.float64))
        half = (mpmath.log(mpmath.mpf(const.P) - 1, 2) + 5) / 2
        for t, i in enumerate(st["rows"]):
            if st["rmax"][t] == 0:
                continue
            alpha = int(np.frexp(A64[i].max())[1]) - 1
            ap = alpha + mpmath.log(int(st["rmax"][t]), 2) / 2
            if st["mu"][t] < -ap + half:
                bad.append(f"Lemma 1 violated for mu at row {i}")
        for t, j in enumerate(st["cols"]):
            if st["cmax"][t] == 0:
                continue
            beta = int(np.frexp(B64[:, j].max())[1]) - 1
            bp = beta + mpmath.log(int(st["cmax"][t]), 2) / 2
            if st["nu"][t] < -bp + half:
                bad.append(f"Lemma 1 violated for nu at col {j}")
    return bad


def pin_residues(st):
    """Theorem CRT: W_l == A'B' (mod p_l) entrywise, residues in the symmetric
    INT8 range, and the integer CRT sum_l x_l W_l reduced into (-P/2, P/2]
    reproduces A'B' exactly (unique by Lemma 0)."""
    bad = []
    const = st["const"]
    ApBp = st["Ap"].dot(st["Bp"])
    acc = np.zeros(ApBp.shape, dtype=object)
    for l, p in enumerate(const.p):
        for name, X in (("A'_l", st["Al"][l]), ("B'_l", st["Bl"][l]), ("W_l", st["W"][l])):
            lo, hi = (-128, 127) if p == 256 else (-(p // 2), p // 2)
            if X.size and (X.min() < lo or X.max() > hi):
                bad.append(f"{name} out of the symmetric range for p={p}")
        if np.any(np.mod(st["Al"][l].astype(object) - st["Ap"], p) != 0):
            bad.append(f"A'_l != A' mod {p}")
        if np.any(np.mod(st["W"][l].astype(object) - ApBp, p) != 0):
            bad.append(f"W_l != A'B' mod {p}")
        acc = acc + st["W"][l].astype(object) * const.x[l]
    P = const.P
    red = np.vectorize(lambda v: ((v + P // 2) % P) - P // 2 if P % 2 == 0 else ((v + (P - 1) // 2) % P) - (P - 1) // 2,
                       otypes=[object])(acc)
    if np.any(red != ApBp):
        bad.append("integer CRT reconstruction != A'B'")
    return bad


def pin_accumulation(st):
    """Lemma 2 (accumulation), Lemma 3 (Q exact), Lemma 4 (final reduction);
    for b=64 also that C'(1) summed in reverse order in FP64 is unchanged
    (it is exact, Lemma 2)."""
    bad = []
    const = st["const"]
    W = st["W"]
    N, rho, P = const.N, const.rho, const.P
    Cex = np.zeros(W[0].shape, dtype=object)
    Qex_num = np.zeros(W[0].shape, dtype=object)
    for l in range(N):
        Cex = Cex + W[l].astype(object) * const.x[l]
    ApBp = st["Ap"].dot(st["Bp"])
    if const.b == 64:
        rev = np.zeros(W[0].shape)
        for l in reversed(range(N)):
            rev = rev + const.s1[l] * W[l].astype(np.float64)
        if np.any(rev != st["C1"]):
            bad.append("C'(1) is not exact (reverse-order FP64 sum differs)")
        lim2 = Fraction(2) ** (1 + const.clog2rho) * (N + 1 + N * U64) * U64 ** 2 * rho * P
    else:
        lim2 = (N + 1) * U64 * rho * P
    R = R_const(const)
    for idx in np.ndindex(W[0].shape):
        got = Fraction(float(st["C1"][idx])) + (Fraction(float(st["C2"][idx])) if const.b == 64 else 0)
        if abs(got - Cex[idx]) > lim2:
            bad.append(f"Lemma 2 bound violated at {idx}")
            break
        qex = sum(Fraction(const.q[l], const.p[l]) * int(W[l][idx]) for l in range(N))
        fl = qex.numerator // qex.denominator
        rnd = fl + (1 if qex - fl > Fraction(1, 2) else 0)   # exact ties impossible (Lemma 0)
        if float(rnd) != st["Q"][idx]:
            bad.append(f"Lemma 3 violated: Q != Q_exact at {idx}")
            break
        if abs(int(ApBp[idx]) - Fraction(float(st["Cpp"][idx]))) > R + R_rel(const) * abs(int(ApBp[idx])):
            bad.append(f"Lemma 4 violated at {idx}")
            break
    return bad


def pin_theorem1(A, B, st):
    """Theorem 1: |AB - C| <= est1 <= est2 entrywise, with exact AB."""
    bad = []
    ApBp = st["Ap"].dot(st["Bp"])
    est1, est2 = theorem1(A, B, st, ApBp)
    AB = exact_product(A.astype(np.float64), B.astype(np.float64), st["rows"], st["cols"])
    err = abs_error(st["C"].astype(np.float64), AB)
    for idx in np.ndindex(err.shape):
        if mpmath.mpf(err[idx]) > est1[idx]:
            bad.append(f"Theorem 1 violated: err > est1 at {idx}")
            break
        if est1[idx] > est2[idx]:
            bad.append(f"est1 > est2 at {idx}")
            break
    return bad


def all_pins(A, B, st):
    return (pin_scaling(A, B, st) + pin_lemma0_lemma1(A, B, st) + pin_residues(st)
            + pin_accumulation(st) + pin_theorem1(A, B, st))


# --------------------------------------------------------------------------
# Algorithm 2's scalar steps: Dbar = single_up(Cbar) and e = log2f(Dbar)
# --------------------------------------------------------------------------


def single_up_reference(M: np.ndarray) -> np.ndarray:
    """Round-up of nonnegative integers to FP32 computed with numpy's own
    conversion: float32(M) rounds to nearest, and one step toward +inf fixes
    the values it rounded down.  Independent of the oracle's exact-rational
    rounding helper."""
    M = np.asarray(M, dtype=np.int64)
    f = M.astype(np.float32)
    low = f.astype(np.float64) < M.astype(np.float64)   # exact: M < 2^53
    f[low] = np.nextafter(f[low], np.float32(np.inf))
    return f.astype(np.int64)


def single_up_cases(seed: int = 0) -> np.ndarray:
    """Every M in [0, 2^12] and (2^24, 2^24 + 2^12], powers of two and their
    neighbours up to 2^32, the values one above and one below each FP32 value
    near 2^25..2^32, and 10^5 random M up to 2^29 plus 10^4 up to 2^32."""
    rng = np.random.default_rng(seed)
    parts = [np.arange(0, 2 ** 12 + 1), np.arange(2 ** 24 + 1, 2 ** 24 + 2 ** 12 + 1)]
    pw = np.array([2 ** e for e in range(33)], dtype=np.int64)
    parts += [pw, pw - 1, pw + 1]
    for e in range(25, 33):
        grid = 2 ** (e - 24)                       # FP32 spacing in [2^(e-1), 2^e)
        base = rng.integers(2 ** (e - 1) // grid, 2 ** e // grid, 200) * grid
        parts += [base, base + 1, base - 1]
    parts += [rng.integers(1, 2 ** 29 + 1, 10 ** 5), rng.integers(1, 2 ** 32, 10 ** 4)]
    M = np.concatenate(parts).astype(np.int64)
    return M[(M >= 0) & (M <= 2 ** 32)]


def pin_single_up(fn, M: np.ndarray) -> list:
    """fn (the oracle's single_up_int or a planted variant) against
    single_up_reference on every M; returns failure strings."""
    ref = single_up_reference(M)
    bad = []
    for x, r in zip(M.tolist(), ref.tolist()):
        if fn(int(x)) != r:
            bad.append(f"single_up({x}) = {fn(int(x))}, expected {r}")
            if len(bad) > 5:
                break
    return bad


def log2f_near_midpoint_inputs(lo: int, hi: int) -> np.ndarray:
    """Integer-valued FP32 d in [lo, hi] whose FP64 log2 lies within 2^-40
    (relative) of an FP32 rounding midpoint: exactly the inputs the oracle's
    vectorised log2f settles one by one."""
    out = []
    for a in range(lo, hi + 1, 1 << 22):
        d = np.arange(a, min(a + (1 << 22), hi + 1), dtype=np.float64)
        d = d[d.astype(np.float32).astype(np.float64) == d]          # FP32 values only
        v = np.log2(d)
        r = v.astype(np.float32)
        up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
        dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
        rd = r.astype(np.float64)
        tol = np.abs(v) * 2.0 ** -40
        near = (np.abs(v - 0.5 * (rd + up)) <= tol) | (np.abs(v - 0.5 * (rd + dn)) <= tol)
        out.append(d[near])
    return np.concatenate(out) if out else np.zeros(0)


def pin_log2f_many(fn, d: np.ndarray) -> list:
    """fn (the oracle's log2f_many or a planted variant) against the
    decimal-pinned scalar log2f, element by element."""
    from oracle.ozaki2 import log2f
    got = fn(np.asarray(d, dtype=np.float32))
    bad = []
    for x, g in zip(np.asarray(d).tolist(), got.tolist()):
        ref = float(log2f(int(x)))
        if float(np.float32(ref)) != g:
            bad.append(f"log2f_many({int(x)}) = {g!r}, expected {ref!r}")
            if len(bad) > 5:
                break
    return bad


# --------------------------------------------------------------------------
# k beyond 2^17 (reading R22): inputs that push a residue product past INT32
# --------------------------------------------------------------------------


def fold_inputs(m: int, n: int, k: int, N: int, p: int = 255, seed: int = 0):
    """Constant rows of A and columns of B whose scaled integers are all
    congruent to (p - 1)/2 modulo the odd modulus p, so that every term of
    the residue product modulo p is ((p - 1)/2)^2 and the product reaches
    k ((p - 1)/2)^2: beyond 2^31 for k >= 2^18 at p = 255.  Built with the
    oracle's own scaling: with every entry 2^-5 * 47.5 = 1.484375 (Abar = 48,
    far from a ceiling step) the shift mu is found, then the entry is moved
    by less than p units of 2^-mu to the nearest integer of that class, which
    leaves mu', Abar and hence mu unchanged.  Random signs per row / column
    keep the sign pattern from cancelling.  Needs 2^mu < 2^53 (small N)."""
    from oracle.constants import constants
    from oracle.ozaki2 import scaling

    rng = np.random.default_rng(seed)
    base = 1.484375
    probeA, probeB = np.full((1, k), base), np.full((k, 1), base)
    st = scaling(probeA, probeB, N)
    assert p in constants(N).p
    want = (p - 1) // 2

    def moved(shift):
        X = int(Fraction(base) * Fraction(2) ** int(shift))
        X += (want - X) % p
        assert X < 2 ** 53
        return float(Fraction(X) / Fraction(2) ** int(shift))

    a, b = moved(st["mu"][0]), moved(st["nu"][0])
    sa = rng.choice([-1.0, 1.0], (m, 1))
    sb = rng.choice([-1.0, 1.0], (1, n))
    A = np.full((m, k), a) * sa
    B = np.full((k, n), b) * sb
    return A, B
