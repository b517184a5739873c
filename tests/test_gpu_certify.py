"""GPU parity of the a-posteriori certified call (ozaki2_gemm_certified).

The library evaluates Theorem 1's est1 after each run, with |A'B'| bounded
through Lemma 4 by the computed C'' and S = |A||B| replaced by its certified
BF16 lower bound, every rounding upward.  Since C (hence C'') is bit-identical
to the oracle's, the GPU's ratio max est1/S lies between the oracle's (exact
S) and the oracle's divided by the lower bound's accuracy factor.  The N it
settles on is therefore at least the oracle's minimal certified N for eps and
at most the oracle's for eps (1 - DELTA(k)).
"""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.bounds import certified_moduli, certified_ratio, required_moduli
from oracle.ozaki2 import os_ii
from workload import gemm_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


def delta(k):
    # S_lower >= S (1 - 2^-6) (1 - k 2^-22); a few upward roundings on top
    return 1.0 - (1.0 - 2.0 ** -6) * (1.0 - k * 2.0 ** -22) + 1e-9


@pytest.mark.parametrize("m,n,k,N,phi,dtype", [
    (100, 90, 300, 14, 0.5, np.float64),
    (70, 65, 200, 20, 2.0, np.float64),
    (60, 50, 150, 49, 4.0, np.float64),
    (64, 50, 150, 7, 0.5, np.float32),
    (40, 30, 6000, 14, 1.0, np.float64),    # small output, long k: split residue products
])
def test_certified_ratio_at_fixed_N(m, n, k, N, phi, dtype):
    announce(f"certified ratio m={m} n={n} k={k} N={N} phi={phi} {np.dtype(dtype).name}")
    A, B = gemm_inputs(m, n, k, phi=phi, seed=m + N, dtype=dtype)
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), 1.0, N)   # eps = 1: the first N passes
    assert rc == oz.OK and N_used == N
    C_ref, st = os_ii(A, B, N, stages=True)
    assert np.array_equal(host(C), C_ref)
    want = certified_ratio(A, B, st)
    assert want * (1 - 1e-12) <= ratio <= want / (1 - delta(k)), (ratio, want)


@pytest.mark.parametrize("phi,eps,dtype", [(0.5, 1e-14, np.float64), (2.0, 1e-14, np.float64),
                                           (1.0, 1e-12, np.float64), (0.5, 1e-6, np.float32)])
def test_certified_adaptive_N(phi, eps, dtype):
    m, n, k = 60, 50, 200
    announce(f"certified adaptive phi={phi} eps={eps} {np.dtype(dtype).name}")
    A, B = gemm_inputs(m, n, k, phi=phi, seed=7 + int(phi), dtype=dtype)
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), eps)
    assert rc == oz.OK and ratio <= eps
    # the oracle's minimal certified N (no certified N lies below the planner's)
    N0, _, _ = required_moduli(A, B, eps)
    lo, ok_lo, _ = certified_moduli(A, B, eps, N0)
    N1, _, _ = required_moduli(A, B, eps * (1 - delta(k)))
    hi, ok_hi, _ = certified_moduli(A, B, eps * (1 - delta(k)), N1)
    assert ok_lo and ok_hi and lo <= N_used <= hi, (lo, N_used, hi)
    assert np.array_equal(host(C), host(oz.gemm(dev(A), dev(B), N_used)))


def test_certified_explicit_start_and_unreachable():
    announce("certified: explicit start, unreachable target")
    A, B = gemm_inputs(40, 30, 80, phi=1.0, seed=3)
    # an explicit start above the needed N is kept
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), 1e-12, 30)
    assert rc == oz.OK and N_used == 30 and ratio <= 1e-12
    # output rounding alone exceeds 1e-17 |A||B|: every N up to 49 is tried
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), 1e-17, 45)
    assert rc == oz.ERR_UNREACHABLE and N_used == 49 and ratio > 1e-17
    assert np.array_equal(host(C), os_ii(A, B, 49))
    # FP32 stops at 16
    Af, Bf = A.astype(np.float32), B.astype(np.float32)
    C, rc, N_used, ratio = oz.gemm_certified(dev(Af), dev(Bf), 1e-12, 14)
    assert rc == oz.ERR_UNREACHABLE and N_used == 16
    assert oz.ozaki2_sync_status() == oz.OK


def test_certified_nonfinite_and_k0():
    announce("certified: non-finite input, k = 0")
    A, B = gemm_inputs(30, 20, 40, phi=1.0, seed=4)
    A[3, 5] = np.inf
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), 1e-14)
    assert rc == oz.ERR_NONFINITE
    assert np.all(np.isnan(host(C)))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert oz.ozaki2_sync_status() == oz.OK
    Z = torch.zeros((5, 0), dtype=torch.float64, device="cuda:0")
    C, rc, N_used, ratio = oz.gemm_certified(Z, torch.zeros((0, 4), dtype=torch.float64, device="cuda:0"), 1e-14)
    assert rc == oz.OK and ratio == 0.0 and torch.all(C == 0).item()


def test_certified_caller_owned_workspace():
    # A caller-installed workspace of exactly ozaki2_certified_workspace_bytes
    # at the N used is enough (same bits as on the library's); one byte less
    # is refused before anything runs.
    announce("certified: caller-owned workspace")
    A, B = gemm_inputs(70, 60, 90, phi=1.0, seed=8)
    ref, rc, N, _ = oz.gemm_certified(dev(A), dev(B), 1.0, 18)
    assert rc == oz.OK and N == 18
    ref = host(ref)
    try:
        nbytes = oz.ozaki2_certified_workspace_bytes(64, 70, 60, 90, 18)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        assert oz.ozaki2_set_workspace(ws.data_ptr(), nbytes) == oz.OK
        C, rc, N, _ = oz.gemm_certified(dev(A), dev(B), 1.0, 18)
        assert rc == oz.OK and N == 18 and np.array_equal(host(C), ref)
        assert oz.ozaki2_set_workspace(ws.data_ptr(), nbytes - 1) == oz.OK
        _, rc, _, _ = oz.gemm_certified(dev(A), dev(B), 1.0, 18)
        assert rc == oz.ERR_WORKSPACE
        torch.cuda.synchronize()
    finally:
        oz.ozaki2_set_workspace(None, 0)


def test_certified_tiny_nonzero_entry_is_not_skipped():
    # Entry (0, 1) of |A||B| is 2^-160 > 0, but its lower bound underflows to
    # 0.  It must not be skipped: the certificate is infinite at every N and
    # the call ends UNREACHABLE at N = 49, with C the plain result at 49.
    announce("certified: nonzero entry whose lower bound of S underflows")
    A, B = gemm_inputs(60, 70, 90, phi=0.5, seed=41)
    A[0, :] = 0.0
    A[0, 0], A[0, 2] = 1.0, 2.0 ** -80
    B[:, 1] = 0.0
    B[1, 1], B[2, 1] = 1.0, 2.0 ** -80
    C, rc, N_used, ratio = oz.gemm_certified(dev(A), dev(B), 1e-3, 40)
    assert rc == oz.ERR_UNREACHABLE and N_used == 49 and ratio == float("inf")
    assert np.array_equal(host(C), os_ii(A, B, 49))
