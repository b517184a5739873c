"""Pins of the oracle's algorithm (Algorithms 1-3) against the paper's lemmas,
Theorem 1 and plain mathematics, on tiny seeded inputs for every N."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.ozaki2 import os_ii
from pins import (all_pins, fold_inputs, pin_accumulation, pin_lemma0_lemma1, pin_residues,
                  pin_scaling, pin_theorem1)
from workload import gemm_inputs, wrap_inputs


@pytest.mark.parametrize("N", list(range(2, 50)))
def test_all_pins_fp64_every_N(N):
    A, B = gemm_inputs(5, 4, 7, phi=1.0, seed=N)
    _, st = os_ii(A, B, N, stages=True)
    assert all_pins(A, B, st) == []


@pytest.mark.parametrize("N", list(range(2, 17)))
def test_all_pins_fp32_every_N(N):
    A, B = gemm_inputs(5, 4, 7, phi=1.0, seed=100 + N, dtype=np.float32)
    _, st = os_ii(A, B, N, stages=True)
    assert all_pins(A, B, st) == []


def test_int32_wrap_at_k_max():
    # k = 2^17 (the largest k of the analysis) with every residue of A' and B'
    # modulo 256 equal to -128 (N = 14 for these inputs): each of the k terms
    # of the p = 256 residue product is 2^14, so the INT32 sum is 2^31 and
    # wraps to -2^31.  Wrap-around keeps it congruent mod 256 (W = 0), which
    # Theorem CRT needs; every lemma and Theorem 1 must still hold.
    A, B = wrap_inputs(4, 3, 2 ** 17, seed=1)
    _, st = os_ii(A, B, 14, stages=True)
    l = list(st["const"].p).index(256)
    assert np.all(st["Al"][l] == -128) and np.all(st["Bl"][l] == -128)
    assert np.all(st["Cl"][l] == -2 ** 31)
    assert np.all(st["W"][l] == 0)
    assert all_pins(A, B, st) == []


@pytest.mark.parametrize("phi", [0.0, 1.0, 4.0])
@pytest.mark.parametrize("N", [6, 14, 20])
def test_pins_wider(phi, N):
    A, B = gemm_inputs(12, 9, 40, phi=phi, seed=int(phi * 10) + N)
    _, st = os_ii(A, B, N, stages=True)
    assert all_pins(A, B, st) == []


def test_paper_setup_reduced():
    # Section 5 setup (A, B ~ (rand-0.5) exp(phi randn)) at reduced size,
    # FP64 and FP32: observed error never exceeds est1 (Theorem 1).
    for dt, N in ((np.float64, 12), (np.float32, 6)):
        A, B = gemm_inputs(16, 16, 256, phi=2.0, seed=3, dtype=dt)
        _, st = os_ii(A, B, N, stages=True)
        assert pin_theorem1(A, B, st) == []


def test_integer_inputs_are_exact():
    # Integer inputs whose scaled copies stay integer (mu, nu >= 0) have no
    # truncation error; with |A'B'| < 2^53 every CRT step is exact, so C == AB.
    rng = np.random.default_rng(11)
    A = rng.integers(-20, 21, (7, 6)).astype(np.float64)
    B = rng.integers(-20, 21, (6, 5)).astype(np.float64)
    for N in (4, 5, 6):
        C, st = os_ii(A, B, N, stages=True)
        assert np.all(st["mu"] >= 0) and np.all(st["nu"] >= 0)
        assert np.array_equal(C, A @ B)


def test_zero_rows_and_columns_give_exact_zeros():
    A, B = gemm_inputs(6, 5, 8, seed=5)
    A[2, :] = 0.0
    B[:, 3] = 0.0
    A[4, :4] = 0.0
    B[4:, 1] = 0.0          # row 4 of A and column 1 of B have disjoint supports
    C, st = os_ii(A, B, 14, stages=True)
    assert np.all(C[2, :] == 0) and np.all(C[:, 3] == 0) and C[4, 1] == 0
    assert pin_residues(st) == [] and pin_accumulation(st) == []


def test_scalar_closed_form():
    # m = n = k = 1: Abar = ceil(2^mu'|a|) in [32, 64], Cbar = Abar*Bbar, and
    # the result is a*b up to the Lemma 4 rounding (3u relative) once the
    # truncation vanishes (N >= 16 keeps every bit of a and b).
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b = rng.standard_normal(2) * np.exp(rng.standard_normal(2) * 3)
        C, st = os_ii(np.array([[a]]), np.array([[b]]), 20, stages=True)
        assert 32 * 32 <= st["rmax"][0] <= 64 * 64
        exact = Fraction(float(a)) * Fraction(float(b))
        assert abs(Fraction(float(C[0, 0])) - exact) <= 4 * Fraction(1, 2 ** 53) * abs(exact)


def test_n2_bruteforce():
    # N = 2 (P = 65280): A'B' is small enough to check every stage by brute force.
    A, B = gemm_inputs(3, 3, 4, seed=9)
    _, st = os_ii(A, B, 2, stages=True)
    assert st["const"].P == 256 * 255
    assert pin_scaling(A, B, st) == [] and pin_lemma0_lemma1(A, B, st) == []
    assert pin_residues(st) == [] and pin_accumulation(st) == []


def test_row_col_subset_matches_full():
    # The sampled-entry form used at full size must agree with the full run.
    A, B = gemm_inputs(20, 18, 30, phi=1.0, seed=4)
    C = os_ii(A, B, 13)
    rows, cols = [0, 7, 19], [3, 17]
    Cs = os_ii(A, B, 13, rows=rows, cols=cols)
    assert np.array_equal(Cs, C[np.ix_(rows, cols)])


def test_domain_errors():
    A, B = gemm_inputs(3, 3, 3)
    A[1, 1] = np.inf
    with pytest.raises(ValueError):
        os_ii(A, B, 10)
    A, B = gemm_inputs(3, 3, 3, dtype=np.float32)
    with pytest.raises(ValueError):
        os_ii(A, B, 17)
    assert os_ii(np.zeros((3, 0)), np.zeros((0, 2)), 10).shape == (3, 2)


@pytest.mark.parametrize("k", [2 ** 17 + 1, 2 ** 18])
def test_k_beyond_2_17_pins(k):
    # Reading R22: k up to 2^19 - 1.  Random inputs: every lemma and
    # Theorem 1 hold, and Cbar stays below 2^12 k < 2^31.
    A, B = gemm_inputs(3, 2, k, phi=1.0, seed=k % 1000)
    _, st = os_ii(A, B, 14, stages=True)
    assert all_pins(A, B, st) == []


def test_k_beyond_2_17_residue_product_past_int32():
    # Every term of the p = 255 residue product is 127^2, so at k = 2^18 the
    # product is 2^18 127^2 > 2^31: one INT32 accumulation over all of k
    # would wrap (and 2^32 = 1 mod 255, so W would be off by one).  The
    # chunked accumulation of reading R22 keeps W = A'B' mod p exactly.
    k = 2 ** 18
    A, B = fold_inputs(2, 3, k, 14)
    _, st = os_ii(A, B, 14, stages=True)
    l = list(st["const"].p).index(255)
    assert np.all(np.abs(st["Al"][l]) == 127) and np.all(np.abs(st["Bl"][l]) == 127)
    assert np.all(np.abs(st["Cl"][l]) == k * 127 * 127) and k * 127 * 127 >= 2 ** 31
    assert all_pins(A, B, st) == []


def test_largest_k():
    # k = 2^19 - 1, the largest k accepted: Cbar <= 2^12 k < 2^31.
    k = 2 ** 19 - 1
    A, B = gemm_inputs(2, 2, k, phi=0.5, seed=3)
    _, st = os_ii(A, B, 12, stages=True)
    assert st["rmax"].max() < 2 ** 31
    assert pin_residues(st) == [] and pin_lemma0_lemma1(A, B, st) == []
    with pytest.raises(ValueError):
        os_ii(np.ones((1, 2 ** 19)), np.ones((2 ** 19, 1)), 12)
