"""GPU parity of the complex calls (ozaki2_zgemm / ozaki2_cgemm, reading
R23: the real method on the real embedding) against the complex oracle:
every output entry bit-identical, on ragged shapes spanning several tiles,
both moduli tables, k = 0, and a non-finite entry.  At 4096^3 sampled
rows x columns are compared."""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.complex_gemm import os_ii_complex
from workload import complex_gemm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


@pytest.mark.parametrize("m,n,k,N,phi,dt", [
    (300, 200, 250, 14, 0.5, np.complex128),   # 2m x n x 2k = 600 x 200 x 500
    (1, 1, 1, 7, 0.5, np.complex128),
    (129, 70, 65, 20, 2.0, np.complex128),
    (64, 257, 100, 49, 1.0, np.complex128),
    (65, 33, 256, 28, 1.0, np.complex128),    # three limbs; k a multiple of 128
    (40, 35, 129, 36, 0.5, np.complex128),    # three exact steps; k just past 128
    (70, 20, 300, 2, 0.5, np.complex128),
    (200, 150, 130, 7, 0.5, np.complex64),
    (33, 40, 300, 16, 1.0, np.complex64),
])
def test_zgemm_matches_oracle(m, n, k, N, phi, dt):
    announce(f"complex m={m} n={n} k={k} N={N} {np.dtype(dt).name}")
    A, B = complex_gemm_inputs(m, n, k, phi=phi, seed=m + n + k + N, dtype=dt)
    got = host(oz.zgemm(dev(A), dev(B), N))
    want = os_ii_complex(A, B, N)
    assert got.dtype == want.dtype
    assert np.array_equal(got, want), f"{int(np.sum(got != want))} of {got.size} differ"
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm_optimal_table():
    announce("complex with the optimal moduli table")
    A, B = complex_gemm_inputs(90, 80, 70, phi=1.0, seed=3)
    with oz.moduli_table(oz.MODULI_OPTIMAL):
        got = host(oz.zgemm(dev(A), dev(B), 14))
    assert np.array_equal(got, os_ii_complex(A, B, 14, table="optimal"))


def test_zgemm_edge_cases():
    announce("complex edge cases: leading dimensions, k = 0, non-finite")
    m, n, k, N = 50, 40, 60, 12
    A, B = complex_gemm_inputs(m, n, k, phi=1.0, seed=8)
    lda, ldb, ldc = m + 3, k + 2, m + 5
    Abuf = np.full((k, lda), np.nan + 1j * np.nan)
    Abuf[:, :m] = A.T
    Bbuf = np.full((n, ldb), np.nan + 1j * np.nan)
    Bbuf[:, :k] = B.T
    dA, dB = dev(Abuf), dev(Bbuf)
    dC = torch.full((n, ldc), 7.0 + 0j, dtype=torch.complex128, device="cuda:0")
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    assert oz.ozaki2_zgemm(m, n, k, dA.data_ptr(), lda, dB.data_ptr(), ldb, dC.data_ptr(), ldc, N) == oz.OK
    Cbuf = host(dC)
    assert np.all(Cbuf[:, m:] == 7.0)
    assert np.array_equal(Cbuf[:, :m].T, os_ii_complex(A, B, N))
    # k = 0 writes zeros
    Z = oz.zgemm(torch.zeros((5, 0), dtype=torch.complex128, device="cuda:0"),
                 torch.zeros((0, 4), dtype=torch.complex128, device="cuda:0"), 10)
    assert torch.all(Z == 0).item()
    # a non-finite imaginary part: every output NaN and the status set
    A[3, 4] = 1.0 + 1j * np.inf
    got = host(oz.zgemm(dev(A), dev(B), N))
    assert np.all(np.isnan(got.real)) and np.all(np.isnan(got.imag))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm_4096_sampled():
    m = n = k = 4096
    N = 16
    announce(f"complex {m}^3 N={N} sampled")
    A, B = complex_gemm_inputs(m, n, k, phi=0.5, seed=0)
    got = host(oz.zgemm(dev(A), dev(B), N))
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(m, 6, replace=False))
    cols = np.sort(rng.choice(n, 6, replace=False))
    assert np.array_equal(got[np.ix_(rows, cols)], os_ii_complex(A, B, N, rows=rows, cols=cols))
    assert oz.ozaki2_sync_status() == oz.OK


def test_zgemm_captured_in_a_graph():
    # ozaki2_zgemm enqueues kernels only; after a first call has grown the
    # workspace it can be captured and replayed, each replay giving the eager
    # call's bits (other work and a reset of C between replays).
    announce("ozaki2_zgemm captured in a graph")
    m, n, k, N = 200, 150, 120, 13
    A, B = complex_gemm_inputs(m, n, k, phi=1.0, seed=12)
    ref = host(oz.zgemm(dev(A), dev(B), N))
    dA, dB = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    C = torch.full((n, m), float("nan"), dtype=torch.complex128, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc = oz.ozaki2_zgemm(m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, C.data_ptr(), m, N)
    assert rc == oz.OK
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    for rep in range(2):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C).T, ref), f"replay {rep}"
        X, Y = complex_gemm_inputs(40, 30, 50, seed=60 + rep)
        assert np.array_equal(host(oz.zgemm(dev(X), dev(Y), 10)), os_ii_complex(X, Y, 10))
