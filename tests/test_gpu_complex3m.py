"""GPU parity of the complex 3-product calls (ozaki2_zgemm3m /
ozaki2_cgemm3m, reading R25: shared shifts per complex row and column,
three residue products per modulus) against the oracle's
os_ii_complex_3m: every output entry bit-identical on ragged shapes that
span several tiles, both moduli tables, leading dimensions, k = 0, a
non-finite entry and k beyond 2^18 (which the embedding cannot take).  At
4096^3 sampled rows x columns are compared."""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.complex_gemm import os_ii_complex_3m
from workload import complex_gemm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


@pytest.mark.parametrize("m,n,k,N,phi,dt", [
    (300, 130, 150, 14, 0.5, np.complex128),
    (1, 1, 1, 7, 0.5, np.complex128),
    (129, 70, 65, 20, 2.0, np.complex128),
    (64, 257, 60, 49, 1.0, np.complex128),
    (260, 33, 700, 2, 0.5, np.complex128),
    (70, 50, 90, 28, 1.0, np.complex128),
    (40, 35, 130, 36, 0.5, np.complex128),
    (200, 150, 130, 7, 0.5, np.complex64),
    (33, 40, 300, 16, 1.0, np.complex64),
])
def test_zgemm3m_matches_oracle(m, n, k, N, phi, dt):
    announce(f"complex 3m m={m} n={n} k={k} N={N} {np.dtype(dt).name}")
    A, B = complex_gemm_inputs(m, n, k, phi=phi, seed=m + n + k + N + 1, dtype=dt)
    got = host(oz.zgemm(dev(A), dev(B), N, form="3m"))
    want = os_ii_complex_3m(A, B, N)
    assert got.dtype == want.dtype
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} of {got.size} differ"
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm3m_optimal_table_and_zero_rows():
    announce("complex 3m with the optimal moduli table, zero rows and columns")
    A, B = complex_gemm_inputs(90, 80, 70, phi=1.0, seed=4)
    A[5, :] = 0
    B[:, 7] = 0
    B[:, 9] = 1e-300 + 0j
    with oz.moduli_table(oz.MODULI_OPTIMAL):
        got = host(oz.zgemm(dev(A), dev(B), 14, form="3m"))
    assert np.array_equal(got, os_ii_complex_3m(A, B, 14, table="optimal"))


def test_zgemm3m_edge_cases():
    announce("complex 3m edge cases: leading dimensions, k = 0, non-finite")
    m, n, k, N = 50, 40, 60, 12
    A, B = complex_gemm_inputs(m, n, k, phi=1.0, seed=9)
    lda, ldb, ldc = m + 3, k + 2, m + 5
    Abuf = np.full((k, lda), np.nan + 1j * np.nan)
    Abuf[:, :m] = A.T
    Bbuf = np.full((n, ldb), np.nan + 1j * np.nan)
    Bbuf[:, :k] = B.T
    dA, dB = dev(Abuf), dev(Bbuf)
    dC = torch.full((n, ldc), 7.0 + 0j, dtype=torch.complex128, device="cuda:0")
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    assert oz.ozaki2_zgemm3m(m, n, k, dA.data_ptr(), lda, dB.data_ptr(), ldb, dC.data_ptr(), ldc,
                             N) == oz.OK
    Cbuf = host(dC)
    assert np.all(Cbuf[:, m:] == 7.0)
    assert np.array_equal(Cbuf[:, :m].T, os_ii_complex_3m(A, B, N))
    Z = oz.zgemm(torch.zeros((5, 0), dtype=torch.complex128, device="cuda:0"),
                 torch.zeros((0, 4), dtype=torch.complex128, device="cuda:0"), 10, form="3m")
    assert torch.all(Z == 0).item()
    A[3, 4] = 1.0 + 1j * np.inf
    got = host(oz.zgemm(dev(A), dev(B), N, form="3m"))
    assert np.all(np.isnan(got.real)) and np.all(np.isnan(got.imag))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm3m_k_beyond_the_embedding():
    # k = 2^18 + 100: the embedding would need 2k >= 2^19; the 3-product form
    # keeps k, and its residue products fold mod p every 2^17 of k.
    m, n, k, N = 5, 3, 2 ** 18 + 100, 9
    announce(f"complex 3m k={k}")
    A, B = complex_gemm_inputs(m, n, k, phi=0.5, seed=21)
    got = host(oz.zgemm(dev(A), dev(B), N, form="3m"))
    assert np.array_equal(got, os_ii_complex_3m(A, B, N))


def test_zgemm3m_accuracy_against_the_embedding():
    # Both forms are accurate to about the same level at large N.
    announce("complex 3m accuracy against the 4-product form")
    A, B = complex_gemm_inputs(120, 110, 500, phi=0.5, seed=30)
    exact = A @ B
    g3 = host(oz.zgemm(dev(A), dev(B), 16, form="3m"))
    g4 = host(oz.zgemm(dev(A), dev(B), 16))
    e3 = np.max(np.abs(g3 - exact)) / np.max(np.abs(exact))
    e4 = np.max(np.abs(g4 - exact)) / np.max(np.abs(exact))
    assert e3 < 1e-13 and e4 < 1e-13


def test_zgemm3m_4096_sampled():
    m = n = k = 4096
    N = 16
    announce(f"complex 3m {m}^3 N={N} sampled")
    A, B = complex_gemm_inputs(m, n, k, phi=0.5, seed=1)
    got = host(oz.zgemm(dev(A), dev(B), N, form="3m"))
    rng = np.random.default_rng(8)
    rows = np.sort(rng.choice(m, 6, replace=False))
    cols = np.sort(rng.choice(n, 6, replace=False))
    want = os_ii_complex_3m(A, B, N, rows=rows, cols=cols)
    assert np.array_equal(got[np.ix_(rows, cols)], want)
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm3m_captured_in_a_graph():
    # ozaki2_zgemm3m enqueues kernels only; after a first call has grown the
    # workspace it can be captured and replayed, each replay giving the eager
    # call's bits (other work and a reset of C between replays).
    announce("ozaki2_zgemm3m captured in a graph")
    m, n, k, N = 200, 150, 120, 13
    A, B = complex_gemm_inputs(m, n, k, phi=1.0, seed=13)
    ref = host(oz.zgemm(dev(A), dev(B), N, form="3m"))
    assert np.array_equal(ref, os_ii_complex_3m(A, B, N))
    dA, dB = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    C = torch.full((n, m), float("nan"), dtype=torch.complex128, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc = oz.ozaki2_zgemm3m(m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, C.data_ptr(), m, N)
    assert rc == oz.OK
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    for rep in range(2):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C).T, ref), f"replay {rep}"
        X, Y = complex_gemm_inputs(40, 30, 50, seed=70 + rep)
        assert np.array_equal(host(oz.zgemm(dev(X), dev(Y), 10, form="3m")),
                              os_ii_complex_3m(X, Y, 10))
