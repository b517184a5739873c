"""Pins of the per-N moduli of largest product (Section 3.1: the set
maximising P depends on N and can be tabulated per N) and of everything the
paper re-derives from the moduli: the constants, the exhaustive claim in the
proof of Lemma 0 for the new P', and Lemmas 0-4 / Theorem 1 on the algorithm
run with those moduli."""
import math
from itertools import combinations

import numpy as np
import pytest

from oracle.constants import MODULI, constants
from oracle.moduli import candidates, optimal_moduli
from oracle.ozaki2 import os_ii
from pins import all_pins
from workload import gemm_inputs

ALL_N = list(range(2, 50))


def brute_force(N):
    """Largest product of N pairwise coprime integers in [2, 256] by plain
    enumeration.  Any set beating the paper's prefix has every element at
    least P_paper / 256^(N-1) (the other N-1 are at most 256 each), so only
    integers from that bound up are enumerated."""
    Pp = math.prod(MODULI[:N])
    lo = -(-Pp // 256 ** (N - 1))
    best, arg = 0, None

    def rec(start, chosen, prod):
        nonlocal best, arg
        if len(chosen) == N:
            if prod > best or (prod == best and tuple(sorted(chosen, reverse=True)) > arg):
                best, arg = prod, tuple(sorted(chosen, reverse=True))
            return
        for v in range(start, 257):
            if all(math.gcd(v, c) == 1 for c in chosen):
                rec(v + 1, chosen + [v], prod * v)

    rec(lo, [], 1)
    return arg


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7])
def test_optimal_moduli_brute_force(N):
    assert optimal_moduli(N) == brute_force(N)


@pytest.mark.parametrize("N", ALL_N)
def test_optimal_moduli_feasible_and_swap_optimal(N):
    p = optimal_moduli(N)
    assert len(p) == N and len(set(p)) == N
    assert all(2 <= v <= 256 for v in p) and list(p) == sorted(p, reverse=True)
    for a, b in combinations(p, 2):
        assert math.gcd(a, b) == 1
    assert math.prod(p) >= math.prod(MODULI[:N])      # the paper's prefix is feasible
    # no single exchange raises P: every integer v <= 256 coprime to the other
    # N - 1 moduli is at most the modulus it would replace
    for i, e in enumerate(p):
        rest = p[:i] + p[i + 1:]
        for v in range(e + 1, 257):
            if v not in p:
                assert any(math.gcd(v, r) != 1 for r in rest), (N, e, v)


def test_255_leaves_the_optimal_set():
    # Section 3.1: the moduli maximising P depend on N, and 255 drops out of
    # them beyond a small N.  The search puts the switch between N = 6 and 7:
    # {249 = 3 * 83, 245 = 5 * 7^2} beats {255, 239} at N = 7, while at N = 6
    # {249, 245} loses to {255, 241} (the paper states it from N >= 6).
    for N in range(2, 7):
        assert optimal_moduli(N) == MODULI[:N]
    for N in range(7, 50):
        assert 255 not in optimal_moduli(N)
    assert 249 * 245 > 255 * 239 and 249 * 245 < 255 * 241


def test_candidate_pruning_is_sound():
    # A dropped v has a larger w <= 256 with every prime factor among v's.
    kept = {v for v, _ in candidates()}
    for v in range(2, 257):
        if v in kept:
            continue
        fv = {q for q in range(2, v + 1) if v % q == 0 and all(q % d for d in range(2, q))}
        assert any(all(q in fv for q in range(2, w + 1) if w % q == 0 and all(q % d for d in range(2, q)))
                   for w in range(v + 1, 257))


@pytest.mark.parametrize("N", ALL_N)
def test_optimal_constants(N):
    # The constants of Section 3.1 for the per-N moduli: CRT inverses, the
    # double-double P, and the s_l1 grid, as for the paper's list.
    from fractions import Fraction
    from oracle.constants import U64
    c = constants(N, 64, "optimal")
    assert c.p == optimal_moduli(N)
    for p, q in zip(c.p, c.q):
        assert 0 < q < p and ((c.P // p) * q) % p == 1
    assert abs(Fraction(c.P1) + Fraction(c.P2) - c.P) <= U64 ** 2 * c.P / 2
    r = max(c.x)
    grid = Fraction(2) ** c.clog2rho * U64 * 2 * 2 ** (r.bit_length() - 1)
    for xl, s1 in zip(c.x, c.s1_int):
        assert Fraction(s1) / grid == int(Fraction(s1) / grid)
        assert 0 <= xl - s1 < Fraction(2) ** (1 + c.clog2rho) * U64 * c.P
    assert c.Pprime >= constants(N, 64).Pprime


@pytest.mark.parametrize("N", ALL_N)
def test_exhaustive_claim_optimal_tables(N):
    # Proof of Lemma 0, re-run for the P' of the per-N moduli: for every
    # integer cbar in [1, 2^16], floor(P' - 0.5(1+u)e') <= P' - 0.5 e' - 2^-21
    # with e' = log2 cbar.  From 2^16 on it holds for any P': 0.5 u e' >= 2^-21
    # there, and floor(y) <= y.
    import mpmath
    pp = float(constants(N, 64, "optimal").Pprime)
    u = 2.0 ** -24
    cb = np.arange(1, 2 ** 16 + 1)
    e = np.log2(cb.astype(np.float64))
    y = pp - 0.5 * (1 + u) * e
    lhs = np.floor(y)
    rhs = pp - 0.5 * e - 2.0 ** -21
    near = (np.abs(y - np.rint(y)) < 1e-9) | (np.abs(lhs - rhs) < 1e-9)
    assert np.all((lhs <= rhs) | near)
    with mpmath.workprec(200):
        for v in cb[near]:
            ev = mpmath.log(int(v), 2)
            l = mpmath.floor(mpmath.mpf(pp) - mpmath.mpf(0.5) * (1 + mpmath.mpf(u)) * ev)
            assert l <= mpmath.mpf(pp) - ev / 2 - mpmath.mpf(2) ** -21


@pytest.mark.parametrize("N", [7, 12, 14, 16, 20, 30, 49])
def test_all_pins_with_optimal_moduli(N):
    # Lemmas 0-4 and Theorem 1 hold for the run with the per-N moduli.
    A, B = gemm_inputs(5, 4, 9, phi=1.0, seed=200 + N)
    _, st = os_ii(A, B, N, stages=True, table="optimal")
    assert st["const"].p == optimal_moduli(N)
    assert all_pins(A, B, st) == []
    if N <= 16:
        A32, B32 = A.astype(np.float32), B.astype(np.float32)
        _, st = os_ii(A32, B32, N, stages=True, table="optimal")
        assert all_pins(A32, B32, st) == []


def test_optimal_moduli_are_never_less_accurate_in_the_bound():
    # P grows, so t = 1/sqrt(32 (P - 1)) shrinks: the planner's N for a target
    # never increases when the per-N moduli replace the paper's prefix.
    from oracle.bounds import planner_terms, required_moduli_from_terms
    A, B = gemm_inputs(12, 10, 60, phi=1.0, seed=3)
    terms = planner_terms(A, B)
    for eps in (1e-10, 1e-13, 1e-15):
        Np = required_moduli_from_terms(terms, eps)
        No = required_moduli_from_terms(terms, eps, 64, "optimal")
        assert No[0] <= Np[0]
