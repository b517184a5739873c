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
