"""Split-k of the single-problem products: when an output has too few tiles
to fill the compute units (small m x n, long k), the scaling product and the
residue products run over k ranges in parallel and a reduction combines the
partial results (the partial mod-p bytes summed mod p; the INT32 partial
sums of Cbar summed before their maxima).  The results must be the same bits
as the unsplit products (OZAKI2_KNOB_SPLIT_K = 1), and match the oracle."""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.complex_gemm import os_ii_complex, os_ii_complex_3m
from oracle.ozaki2 import os_ii
from workload import complex_gemm_inputs, gemm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


def unsplit(f):
    rc, prev = oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, 1)
    assert rc == oz.OK
    try:
        return f()
    finally:
        oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, prev)


@pytest.mark.parametrize("m,n,k,N,dt", [
    (40, 33, 20000, 14, np.float64),          # one 128 x 128 tile, 156 groups of k
    (100, 64, 2 ** 17 + 5, 14, np.float64),   # past 2^17: splits of about 28 groups
    (16, 12, 3 * 2 ** 17, 20, np.float64),
    (130, 129, 9000, 7, np.float32),          # four tiles
    (1, 1, 4096, 2, np.float64),
])
def test_split_matches_unsplit_and_oracle(m, n, k, N, dt):
    announce(f"split-k m={m} n={n} k={k} N={N} {np.dtype(dt).name}")
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=m + n + k, dtype=dt)
    dA, dB = dev(A), dev(B)
    got = host(oz.gemm(dA, dB, N))
    ref = host(unsplit(lambda: oz.gemm(dA, dB, N)))
    assert np.array_equal(got, ref)
    rng = np.random.default_rng(k)
    rows = np.sort(rng.choice(m, min(m, 3), replace=False))
    cols = np.sort(rng.choice(n, min(n, 3), replace=False))
    assert np.array_equal(got[np.ix_(rows, cols)], os_ii(A, B, N, rows=rows, cols=cols))
    assert oz.ozaki2_sync_status() == oz.OK


def test_split_stages_bit_exact():
    # every stage of a split run against the oracle (the stage dump runs the
    # same launch sequence; its INT32 products are taken unsplit)
    from gpu_util import compare_stages
    m, n, k, N = 24, 20, 9000, 13   # residue products split 17 ways, the scaling product 2
    announce(f"split-k stages m={m} n={n} k={k} N={N}")
    A, B = gemm_inputs(m, n, k, phi=2.0, seed=77)
    got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), N).items()}
    C_ref, st = os_ii(A, B, N, stages=True)
    assert compare_stages(got, st, C_ref, N) == []


@pytest.mark.parametrize("form", ["4m", "3m"])
def test_split_complex(form):
    m, n, k, N = 30, 20, 5000, 12
    announce(f"split-k complex {form} m={m} n={n} k={k} N={N}")
    A, B = complex_gemm_inputs(m, n, k, phi=0.5, seed=9)
    dA, dB = dev(A), dev(B)
    got = host(oz.zgemm(dA, dB, N, form=form))
    assert np.array_equal(got, host(unsplit(lambda: oz.zgemm(dA, dB, N, form=form))))
    rows, cols = np.array([0, 17, 29]), np.array([3, 19])
    want = (os_ii_complex_3m if form == "3m" else os_ii_complex)(A, B, N, rows=rows, cols=cols)
    assert np.array_equal(got[np.ix_(rows, cols)], want)
