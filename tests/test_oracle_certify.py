"""Pins of the a-posteriori certification (Theorem 1's est1 with |A'B'| bounded
through Lemma 4 by the computed C'') and of the adaptive choice of N."""
import mpmath
import numpy as np
import pytest

import oracle.bounds as bounds
from oracle.bounds import certified_moduli, certified_ratio, est1_a_posteriori, required_moduli, theorem1
from oracle.exact import abs_error, exact_int_product, exact_product
from oracle.ozaki2 import os_ii
from workload import gemm_inputs


def _check_chain(A, B, N):
    """est1 (exact |A'B'|) <= a-posteriori est1 <= est2 and |AB - C| <= est1 on every entry."""
    C, st = os_ii(A, B, N, stages=True)
    ApBp = exact_int_product(st["Ap"], st["Bp"])
    est1, est2 = theorem1(A, B, st, ApBp)
    post = est1_a_posteriori(A, B, st)
    err = abs_error(C.astype(np.float64), exact_product(A.astype(np.float64), B.astype(np.float64)))
    bad = []
    for idx in np.ndindex(post.shape):
        if not est1[idx] <= post[idx]:
            bad.append(f"a-posteriori est1 below est1 at {idx}")
        if not post[idx] <= est2[idx]:
            bad.append(f"a-posteriori est1 above est2 at {idx}")
        if not mpmath.mpf(err[idx]) <= post[idx]:
            bad.append(f"error above the a-posteriori bound at {idx}")
    return bad


@pytest.mark.parametrize("N,phi,dtype", [(6, 0.5, np.float64), (14, 1.0, np.float64), (20, 4.0, np.float64),
                                         (49, 2.0, np.float64), (5, 0.5, np.float32), (12, 2.0, np.float32)])
def test_a_posteriori_between_est1_and_est2(N, phi, dtype):
    A, B = gemm_inputs(9, 7, 40, phi=phi, seed=N, dtype=dtype)
    assert _check_chain(A, B, N) == []


def test_a_posteriori_with_zero_rows_and_integers():
    # zero rows/columns give exact zeros (bound 0); small integers are exact
    A, B = gemm_inputs(8, 6, 30, phi=1.0, seed=3)
    A[2, :] = 0.0
    B[:, 4] = 0.0
    assert _check_chain(A, B, 14) == []
    _, st = os_ii(A, B, 14, stages=True)
    post = est1_a_posteriori(A, B, st)
    assert all(post[2, j] == 0 for j in range(6)) and all(post[i, 4] == 0 for i in range(8))


# The whole bound includes the output rounding 3 u |A'B'| t^2 2^alpha' 2^beta',
# which exceeds 1e-15 (|A||B|)_ij through the slack of the power-of-two scaling
# (1.5e-15 to 2.6e-15 on these inputs for every N); 1e-14 is certifiable.
@pytest.mark.parametrize("phi,eps,dtype", [(0.5, 1e-14, np.float64), (2.0, 1e-14, np.float64),
                                           (1.0, 1e-12, np.float64), (0.5, 1e-6, np.float32)])
def test_certified_moduli_meets_target_and_is_minimal(phi, eps, dtype):
    A, B = gemm_inputs(10, 8, 60, phi=phi, seed=int(10 * phi), dtype=dtype)
    N0, reach, _ = required_moduli(A, B, eps)
    N, ok, ratio = certified_moduli(A, B, eps, 2)
    assert ok and ratio <= eps
    # the whole-bound certificate can never ask for fewer moduli than the
    # N-dependent part alone (reading R16)
    assert reach and N >= N0
    if N > 2:
        _, st = os_ii(A, B, N - 1, stages=True)
        assert certified_ratio(A, B, st) > eps


def test_certified_moduli_unreachable():
    # the output-rounding part alone is at least 3 u |C''| t^2 2^alpha' 2^beta' > 1e-17 |A||B|
    A, B = gemm_inputs(6, 5, 20, phi=0.5, seed=1)
    N, ok, ratio = certified_moduli(A, B, 1e-17, 40)
    assert not ok and N == 49 and ratio > 1e-17


def test_dropping_the_rounding_term_is_caught(monkeypatch):
    # A planted mistake: the a-posteriori bound without the R_rel |A'B'| term
    # must fall below est1 with the exact |A'B'| somewhere.
    real = bounds._bound_parts

    def no_rel(A, B, st):
        base, tt, Rc, Rr, P, k = real(A, B, st)
        return base, tt, Rc, mpmath.mpf(0), P, k
    A, B = gemm_inputs(9, 7, 40, phi=1.0, seed=5)
    _, st = os_ii(A, B, 14, stages=True)
    ApBp = exact_int_product(st["Ap"], st["Bp"])
    est1, _ = theorem1(A, B, st, ApBp)
    monkeypatch.setattr(bounds, "_bound_parts", no_rel)
    post = est1_a_posteriori(A, B, st)
    assert any(post[idx] < est1[idx] for idx in np.ndindex(post.shape))
