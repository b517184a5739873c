"""Pins of the oracle's constants (Section 3.1) against their defining
properties, computed with tools other than the oracle's own (Python's decimal
module instead of mpmath, integer congruences, exhaustive evaluation)."""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

from oracle.constants import MODULI, U32, U64, beta, constants
from oracle.fp import round_f32
from oracle.ozaki2 import log2f

ALL_N = list(range(2, 50))


def test_moduli_list_shape():
    # Section 3.1: p_l <= 256, pairwise coprime, hence N <= 49; the list is descending.
    assert len(MODULI) == 49
    assert MODULI[0] == 256 and max(MODULI) == 256 and min(MODULI) >= 2
    assert list(MODULI) == sorted(MODULI, reverse=True)
    for a in range(49):
        for b in range(a + 1, 49):
            assert math.gcd(MODULI[a], MODULI[b]) == 1


@pytest.mark.parametrize("N", ALL_N)
def test_inverses_and_crt(N):
    # Theorem CRT / Step 1: (P/p_l) q_l == 1 (mod p_l), 0 < q_l < p_l; and the
    # CRT sum with x_l = (P/p_l) q_l recovers random |x| < P/2 exactly.
    c = constants(N)
    for p, q in zip(c.p, c.q):
        assert 0 < q < p and ((c.P // p) * q) % p == 1
    rng = np.random.default_rng(N)
    for _ in range(20):
        x = int(rng.integers(0, 2 ** 62)) * (c.P // 2 ** 62 + 1) % c.P - c.P // 2
        s = sum(xl * (x % p) for xl, p in zip(c.x, c.p))
        assert ((s - x) % c.P) == 0


@pytest.mark.parametrize("N", ALL_N)
def test_double_double_P(N):
    # eq. (errP): |(P1 + P2) - P| <= u^2 P / 2 and P1 = double(P).
    c = constants(N, 64)
    P1 = int(c.P1)
    ulp = 2 ** (max(P1.bit_length() - 53, 0))
    assert abs(c.P - P1) * 2 <= ulp
    assert abs(Fraction(P1) + Fraction(c.P2) - c.P) <= U64 ** 2 * c.P / 2
    c32 = constants(N, 32)
    assert c32.P2 == 0.0 and c32.P1 == c.P1


@pytest.mark.parametrize("N", ALL_N)
def test_s1_s2_split(N):
    # Section 3.1 and the proof of Lemma 2 (eq. s_i1): s_l1 keeps the upper
    # beta_l bits of x_l, lies on the grid 2^ceil(log2 rho) u 2ufp(r) Z, is
    # below 2 ufp(r), and x_l - s_l1 < 2^(1+ceil(log2 rho)) u P.
    c = constants(N, 64)
    r = max(c.x)
    ufp_r = 2 ** (r.bit_length() - 1)
    grid = Fraction(2) ** c.clog2rho * U64 * 2 * ufp_r
    for xl, s1, s2, bl in zip(c.x, c.s1_int, c.s2, beta(c)):
        assert 0 <= s1 < 2 * ufp_r
        assert Fraction(s1) / grid == int(Fraction(s1) / grid)
        assert 0 <= xl - s1 < Fraction(2) ** (1 + c.clog2rho) * U64 * c.P
        sig = s1 >> ((s1 & -s1).bit_length() - 1) if s1 else 0
        assert sig.bit_length() <= max(bl, 0) or s1 == xl
        # s_l2 = double(x_l - s_l1)
        d = xl - s1
        assert abs(Fraction(s2) - d) <= U64 * d
    assert c.rho == sum(p // 2 for p in c.p)
    assert 2 ** (c.clog2rho - 1) < c.rho <= 2 ** c.clog2rho
    c32 = constants(N, 32)
    assert all(s2 == 0.0 for s2 in c32.s2)
    assert all(abs(Fraction(s) - x) <= U64 * x for s, x in zip(c32.s1, c32.x))


@pytest.mark.parametrize("N", ALL_N)
def test_pprime_with_decimal(N):
    # Algorithm 2: P' = single_down(log2(P-1)/2 - 0.5), re-evaluated with the
    # decimal module (independent of mpmath): P' <= v < P' + ulp(P').
    getcontext().prec = 90
    c = constants(N)
    v = (Decimal(c.P - 1).ln() / Decimal(2).ln()) / 2 - Decimal("0.5")
    pp = c.Pprime
    ulp = Fraction(2) ** (math.floor(math.log2(float(pp))) - 23)
    vf = Fraction(v)
    assert pp <= vf < pp + ulp
    assert round_f32(pp, "rn") == pp
    assert pp < 200            # Section 3.2: P' < 200 for N <= 49


def test_c_constant():
    # single_down(-0.5/(1-4u)) and the two inequalities used in the proofs of
    # Lemma 0 and Lemma 1.
    c = constants(14).c
    assert c == -(Fraction(1, 2) + 3 * Fraction(1, 2 ** 24))
    assert c <= Fraction(-1, 2) * (1 + U32) / (1 - 4 * U32)
    assert c >= Fraction(-1, 2) * (1 + 6 * U32)


@pytest.mark.parametrize("N", ALL_N)
def test_exhaustive_claim(N):
    # Proof of Lemma 0: floor(P' - 0.5(1+u)e') <= P' - 0.5 e' - 2^-21 for
    # e' = log2 cbar.  Checked here for every integer cbar in [1, 2^16] and
    # for 2^16 random cbar in (2^16, 2^29].
    pp = float(constants(N).Pprime)
    u = 2.0 ** -24
    rng = np.random.default_rng(1000 + N)
    cb = np.concatenate([np.arange(1, 2 ** 16 + 1), rng.integers(2 ** 16 + 1, 2 ** 29 + 1, 2 ** 16)])
    e = np.log2(cb.astype(np.float64))
    y = pp - 0.5 * (1 + u) * e
    lhs = np.floor(y)
    rhs = pp - 0.5 * e - 2.0 ** -21
    # float64 evaluation error is < 1e-13 here; flag anything near a decision
    # boundary and settle it in exact arithmetic.
    near = (np.abs(y - np.rint(y)) < 1e-9) | (np.abs(lhs - rhs) < 1e-9)
    assert np.all((lhs <= rhs) | near)
    if near.any():
        import mpmath
        with mpmath.workprec(200):
            for v in cb[near]:
                ev = mpmath.log(int(v), 2)
                l = mpmath.floor(mpmath.mpf(pp) - mpmath.mpf(0.5) * (1 + mpmath.mpf(u)) * ev)
                assert l <= mpmath.mpf(pp) - ev / 2 - mpmath.mpf(2) ** -21


def test_log2f_correctly_rounded_against_decimal():
    # R6: log2f is the round-to-nearest FP32 logarithm; checked against the
    # decimal module for powers of two, their neighbours and random integers.
    getcontext().prec = 60
    rng = np.random.default_rng(7)
    ds = [1, 2, 3, 4, 5, 7, 8, 9, 2 ** 24 - 1, 2 ** 24, 2 ** 24 + 2, 2 ** 29]
    ds += [int(v) for v in rng.integers(1, 2 ** 24, 300)]
    ds += [int(v) << 5 for v in rng.integers(2 ** 19, 2 ** 24, 100)]
    for d in ds:
        got = log2f(d)
        if d & (d - 1) == 0:
            assert got == d.bit_length() - 1
            continue
        v = Fraction(Decimal(d).ln() / Decimal(2).ln())
        ulp = Fraction(2) ** (math.floor(math.log2(float(got))) - 23)
        assert abs(v - got) <= ulp / 2


@pytest.mark.parametrize("table", ["paper", "optimal"])
def test_exhaustive_claim_beyond_2_29(table):
    # Reading R22 (k < 2^19): Cbar can reach 2^31 - 1, so the claim in the
    # proof of Lemma 0 is needed for e' = log2 cbar up to 31.  Above
    # cbar = 2^16 it holds for any P': floor(y) <= y with
    # y = P' - 0.5(1+u)e', and y <= P' - 0.5 e' - 2^-21 once 0.5 u e' >= 2^-21,
    # i.e. e' >= 16.  Checked on every N at 2^16 samples in (2^29, 2^31) and
    # the ends of the range, in exact arithmetic near decision boundaries.
    import mpmath
    u = 2.0 ** -24
    for N in ALL_N:
        pp = float(constants(N, 64, table).Pprime)
        rng = np.random.default_rng(2000 + N)
        cb = np.concatenate([rng.integers(2 ** 29 + 1, 2 ** 31, 2 ** 16),
                             np.array([2 ** 16, 2 ** 29 + 1, 2 ** 31 - 1])])
        e = np.log2(cb.astype(np.float64))
        assert np.all(0.5 * u * e >= 2.0 ** -21)
        y = pp - 0.5 * (1 + u) * e
        lhs, rhs = np.floor(y), pp - 0.5 * e - 2.0 ** -21
        near = (np.abs(y - np.rint(y)) < 1e-9) | (np.abs(lhs - rhs) < 1e-9)
        assert np.all((lhs <= rhs) | near)
        with mpmath.workprec(200):
            for v in cb[near]:
                ev = mpmath.log(int(v), 2)
                lv = mpmath.floor(mpmath.mpf(pp) - mpmath.mpf(0.5) * (1 + mpmath.mpf(u)) * ev)
                assert lv <= mpmath.mpf(pp) - ev / 2 - mpmath.mpf(2) ** -21
