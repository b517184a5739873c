"""Pins of the required-moduli reading (R16) against Theorem 1 and observed
errors: at the N the planner returns, the observed error of the emulation is
within eps * (|A||B|)_ij plus the N-independent rounding part of eq.
(thm:err-2), and one modulus fewer does not meet the target."""
import numpy as np
import pytest
from fractions import Fraction

from oracle.bounds import planner_terms, ratio_max, required_moduli
from oracle.constants import U64
from oracle.exact import exact_product
from oracle.ozaki2 import os_ii
from workload import gemm_inputs


@pytest.mark.parametrize("phi,eps", [(0.5, 1e-13), (1.0, 1e-10), (2.0, 1e-14), (4.0, 1e-12)])
def test_planned_N_meets_target(phi, eps):
    A, B = gemm_inputs(10, 9, 60, phi=phi, seed=int(phi * 7))
    N, ok, det = required_moduli(A, B, eps)
    assert ok and 2 <= N <= 49
    terms = planner_terms(A, B)
    assert ratio_max(terms, N, 64)[0] <= eps
    if N > 2:
        assert ratio_max(terms, N - 1, 64)[0] > eps
    C = os_ii(A, B, N)
    AB = exact_product(A, B)
    S = np.abs(A) @ np.abs(B)
    # N-independent rounding part: (3/2) u P t^2 2^(alpha'+beta') <= (3/64) u (P/(P-1)) ...;
    # bound it by 48 u S * (2^(alpha'+beta') / (2^10 S)) using the planner's own terms.
    amax, bmax = np.abs(A).max(axis=1), np.abs(B).max(axis=0)
    al, be = np.floor(np.log2(amax)), np.floor(np.log2(bmax))
    rnd = (3 / 64) * float(U64) * 1.0001 * np.outer(terms["sr"] * 2.0 ** al, terms["sc"] * 2.0 ** be)
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            err = abs(Fraction(float(C[i, j])) - AB[i, j])
            assert float(err) <= eps * S[i, j] * (1 + 1e-9) + rnd[i, j]


def test_unreachable_target():
    A, B = gemm_inputs(6, 6, 20, phi=1.0, seed=1)
    N, ok, _ = required_moduli(A, B, 1e-40)
    assert not ok and N == 49


def test_wider_exponent_range_needs_more_moduli():
    Ns = [required_moduli(*gemm_inputs(12, 12, 80, phi=phi, seed=3), 1e-15)[0] for phi in (0.0, 4.0)]
    assert Ns[0] <= Ns[1]


def test_entry_whose_S_underflows_admits_no_N():
    # (|A||B|)_ij > 0 with every product term tiny: row [1, 0, 2^-600] of A and
    # column [0, 1, 2^-600] of B give (|A||B|)_01 = 2^-1200, which FP64
    # cannot hold.  That entry is nonzero, so it must not be skipped: no N
    # can meet a relative target for it, and the planner must say so.
    A = np.array([[1.0, 0.0, 2.0 ** -600], [0.5, 0.25, 0.125]])
    B = np.array([[1.0, 0.0], [0.0, 1.0], [0.5, 2.0 ** -600]])
    S_exact = 2.0 ** -600 * 2.0 ** -600
    assert S_exact == 0.0                      # underflows in FP64 ...
    terms = planner_terms(A, B)
    assert terms["nz"][0, 1] and terms["S"][0, 1] == 0.0   # ... but the entry is nonzero
    N, ok, det = required_moduli(A, B, 1e-3)
    assert not ok and N == 49 and det["ratio"] == float("inf")


def test_exact_zero_entries_are_skipped():
    # An entry whose row and column have disjoint supports is exactly zero and
    # does not constrain N.
    A = np.array([[1.0, 0.0], [0.5, 0.25]])
    B = np.array([[0.0, 1.0], [1.0, 0.5]])
    terms = planner_terms(A, B)
    assert not terms["nz"][0, 0] and terms["nz"][0, 1]
    N, ok, _ = required_moduli(A, B, 1e-12)
    assert ok
