"""Cross-implementation pin: the Python oracle (exact rationals, numpy) and
its C++ twin (oracle/os_ii_twin.cpp: plain loops, IEEE double and long
double arithmetic, OpenMP) agree on every stage of Algorithms 1-3, bit for
bit: mu', nu', the Cbar maxima, mu, nu, A'_l, B'_l, W_l, C'(1), C'(2), Q, C''
and C.  The two share only the constants of Section 3.1."""
import numpy as np
import pytest

from oracle.ozaki2 import os_ii
from oracle.twin import os_ii_twin
from workload import gemm_inputs


def compare(A, B, N, table="paper"):
    C_py, sp = os_ii(A, B, N, stages=True, table=table)
    C_tw, st = os_ii_twin(A, B, N, stages=True, table=table)
    bad = []
    for key in ("mu_p", "nu_p", "rmax", "cmax", "mu", "nu"):
        if not np.array_equal(np.asarray(sp[key], dtype=np.int64), st[key].astype(np.int64)):
            bad.append(key)
    for l in range(N):
        if not np.array_equal(np.asarray(sp["Al"][l]), st["Al"][l]):
            bad.append(f"A'_{l}")
        if not np.array_equal(np.asarray(sp["Bl"][l]), st["Bl"][l]):
            bad.append(f"B'_{l}")
        if not np.array_equal(np.asarray(sp["W"][l]), st["W"][l]):
            bad.append(f"W_{l}")
    for key in ("C1", "C2", "Q", "Cpp"):
        if not np.array_equal(sp[key], st[key]):
            bad.append(key)
    if C_py.dtype != C_tw.dtype or not np.array_equal(C_py, C_tw):
        bad.append("C")
    return bad


@pytest.mark.parametrize("N", [2, 5, 7, 12, 14, 16, 20, 23, 31, 32, 40, 49])
def test_twin_fp64(N):
    A, B = gemm_inputs(23, 17, 41, phi=1.0, seed=N)
    assert compare(A, B, N) == []


@pytest.mark.parametrize("N", [2, 7, 11, 16])
def test_twin_fp32(N):
    A, B = gemm_inputs(19, 21, 33, phi=1.0, seed=50 + N, dtype=np.float32)
    assert compare(A, B, N) == []


@pytest.mark.parametrize("phi", [0.0, 2.0, 4.0])
def test_twin_wide_exponents_and_optimal_table(phi):
    A, B = gemm_inputs(30, 20, 60, phi=phi, seed=int(10 * phi))
    A[3, :] = 0.0
    B[:, 5] = 0.0
    A[7, 2] = 5e-320                      # subnormal
    assert compare(A, B, 14) == []
    assert compare(A, B, 20, table="optimal") == []


def test_twin_wrap_and_k_beyond_2_17():
    from pins import fold_inputs
    from workload import wrap_inputs
    A, B = wrap_inputs(3, 2, 2 ** 17, seed=1)          # p = 256 product wraps to -2^31
    assert compare(A, B, 14) == []
    A, B = fold_inputs(2, 2, 2 ** 18, 14)              # p = 255 product beyond 2^31
    assert compare(A, B, 14) == []


def test_twin_rejects_nonfinite():
    A, B = gemm_inputs(4, 4, 4, seed=1)
    A[1, 1] = np.nan
    with pytest.raises(ValueError):
        os_ii_twin(A, B, 10)
