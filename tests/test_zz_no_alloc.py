"""The allocation-free entry point ozaki2_gemm_noalloc, through the C ABI,
against ozaki2_gemm / ozaki2_sgemm on the same inputs: the outputs must be
bit-identical (the same kernels on the same operands; only the workspace
differs), on consecutive calls whose second input is smaller than the
first, so a second call that read what the first left in the scratch array
would show."""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.ozaki2 import os_ii
from workload import gemm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


def _call(entry, prec, A, B, N, fill=float("nan")):
    """C (logical m x n, host) from one call of `entry` ("noalloc" or
    "workspace") on column-major device copies of A and B."""
    m, k = A.shape
    n = B.shape[1]
    dt = torch.float64 if prec == 64 else torch.float32
    Acm, Bcm = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    Ccm = torch.full((n, m), fill, dtype=dt, device="cuda:0")
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    args = (m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(), max(k, 1), Ccm.data_ptr(), max(m, 1), N)
    if entry == "noalloc":
        rc = oz.ozaki2_gemm_noalloc(prec, *args)
    else:
        rc = (oz.ozaki2_gemm if prec == 64 else oz.ozaki2_sgemm)(*args)
    assert rc == oz.OK, (entry, rc)
    return host(Ccm).T


@pytest.mark.parametrize("prec", [64, 32])
def test_noalloc_matches_gemm_on_consecutive_calls(prec):
    dtype = np.float64 if prec == 64 else np.float32
    cases = [(1000, 900, 700, 14 if prec == 64 else 7, 1.0, 5),   # 256 x 256 products
             (300, 200, 500, 9 if prec == 64 else 5, 0.5, 6)]     # smaller, 128 x 128
    for m, n, k, N, phi, seed in cases:
        announce(f"noalloc prec={prec} m={m} n={n} k={k} N={N}")
        A, B = gemm_inputs(m, n, k, phi=phi, seed=seed, dtype=dtype)
        got = _call("noalloc", prec, A, B, N)
        ref = _call("workspace", prec, A, B, N)
        assert np.array_equal(got, ref), f"{int(np.sum(got != ref))} entries differ"
        rows, cols = np.array([0, m // 2, m - 1]), np.array([0, n // 3, n - 1])
        assert np.array_equal(got[np.ix_(rows, cols)], os_ii(A, B, N, rows=rows, cols=cols))
    assert oz.ozaki2_sync_status() == oz.OK


def test_noalloc_split_k():
    # A small output with long k splits its products; the partial results
    # live in the fixed scratch array too.  Two calls in a row, the second
    # smaller (fewer splits), against ozaki2_gemm.
    for m, n, k, N, seed in [(64, 48, 32768, 14, 11), (40, 30, 9000, 10, 12)]:
        announce(f"noalloc split-k m={m} n={n} k={k} N={N}")
        A, B = gemm_inputs(m, n, k, phi=1.0, seed=seed)
        got = _call("noalloc", 64, A, B, N)
        ref = _call("workspace", 64, A, B, N)
        assert np.array_equal(got, ref), f"{int(np.sum(got != ref))} entries differ"
    assert oz.ozaki2_sync_status() == oz.OK


def test_noalloc_edge_cases_and_status():
    announce("noalloc edge cases: k = 0, non-finite input, rejection")
    # k = 0 writes zeros
    got = _call("noalloc", 64, np.zeros((5, 0)), np.zeros((0, 4)), 10)
    assert np.all(got == 0)
    # A non-finite entry: every output NaN, reported once by ozaki2_sync_status
    A, B = gemm_inputs(64, 48, 80, phi=0.5, seed=7)
    A[3, 5] = np.inf
    got = _call("noalloc", 64, A, B, 12, fill=0.0)
    assert np.all(np.isnan(got))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert oz.ozaki2_sync_status() == oz.OK
    # the next call on the same scratch is clean again
    A[3, 5] = 0.25
    assert np.array_equal(_call("noalloc", 64, A, B, 12), _call("workspace", 64, A, B, 12))
    assert oz.ozaki2_sync_status() == oz.OK
    # too large for the scratch array: rejected before anything is enqueued
    Ad = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda:0")
    rc = oz.ozaki2_gemm_noalloc(64, 4096, 4096, 4096, Ad.data_ptr(), 4096, Ad.data_ptr(), 4096,
                                Ad.data_ptr(), 4096, 14)
    assert rc == oz.ERR_WORKSPACE
    assert torch.all(Ad == 0).item()


def test_noalloc_captured_in_a_graph():
    # The callers this entry point is for include code under stream capture:
    # after one call has set up the device's array, a call is captured into a
    # graph and replayed three times, with other allocation-free calls on the
    # same array (which overwrite it) between the replays; every replay must
    # give the eager call's bits.
    announce("noalloc captured in a graph")
    m, n, k, N = 300, 200, 500, 14
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=41)
    ref = _call("noalloc", 64, A, B, N)
    dA, dB = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    C = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc = oz.ozaki2_gemm_noalloc(64, m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, C.data_ptr(), m, N)
    assert rc == oz.OK
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C).T, ref), f"replay {rep}"
        X, Y = gemm_inputs(120, 90, 150, seed=50 + rep)
        assert np.array_equal(_call("noalloc", 64, X, Y, 12), os_ii(X, Y, 12))
    assert oz.ozaki2_sync_status() == oz.OK
