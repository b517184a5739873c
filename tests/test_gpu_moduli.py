"""GPU parity with the per-N moduli of largest product (Section 3.1;
ozaki2_set_moduli_table(OZAKI2_MODULI_OPTIMAL)) against the oracle run
with the same table: every stage bit-exact, the planner's N within the same
bracket as with the paper's list, batched and allocation-free calls equal
to the single call, and the two tables giving different results where their
moduli differ."""
import numpy as np
import pytest

from gpu_util import announce, compare_stages, dev, host
from oracle.bounds import planner_terms, required_moduli_from_terms
from oracle.ozaki2 import os_ii
from workload import gemm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402

OPT = oz.MODULI_OPTIMAL


@pytest.mark.parametrize("m,n,k,N,phi,dt", [
    (300, 200, 500, 14, 0.5, np.float64),    # 255 replaced: 249, 245, 235 among the moduli
    (70, 65, 200, 6, 1.0, np.float64),       # the last N that keeps 255
    (70, 65, 200, 7, 1.0, np.float64),       # the first N without it
    (257, 129, 130, 20, 1.0, np.float64),
    (100, 90, 300, 38, 2.0, np.float64),     # 243 = 3^5 enters
    (70, 65, 200, 49, 4.0, np.float64),
    (768, 1000, 130, 16, 1.0, np.float64),   # 256 x 256 residue products
    (300, 200, 500, 7, 0.5, np.float32),
    (64, 257, 100, 16, 0.5, np.float32),
])
def test_stages_optimal_table(m, n, k, N, phi, dt):
    announce(f"optimal table stages m={m} n={n} k={k} N={N} {np.dtype(dt).name}")
    A, B = gemm_inputs(m, n, k, phi=phi, seed=m + n + k + N, dtype=dt)
    with oz.moduli_table(OPT):
        got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), N).items()}
    C_ref, st = os_ii(A, B, N, stages=True, table="optimal")
    assert compare_stages(got, st, C_ref, N) == []
    assert oz.ozaki2_sync_status() == oz.OK


def test_tables_differ_and_switch_back():
    # N = 14: the two tables differ (255 vs 249, 245, 235), so the results
    # differ somewhere; switching back restores the paper's result exactly.
    announce("optimal table vs paper list, N = 14")
    A, B = gemm_inputs(120, 90, 150, phi=1.0, seed=17)
    dA, dB = dev(A), dev(B)
    paper = host(oz.gemm(dA, dB, 14))
    with oz.moduli_table(OPT):
        opt = host(oz.gemm(dA, dB, 14))
    again = host(oz.gemm(dA, dB, 14))
    assert np.array_equal(paper, os_ii(A, B, 14))
    assert np.array_equal(opt, os_ii(A, B, 14, table="optimal"))
    assert np.array_equal(again, paper)
    assert not np.array_equal(opt, paper)


def test_planner_optimal_table():
    announce("planner with the optimal table")
    from test_gpu_planner import check_between, slack
    for (m, n, k, phi, eps) in [(300, 200, 500, 0.5, 1e-15), (257, 129, 1000, 4.0, 1e-12)]:
        A, B = gemm_inputs(m, n, k, phi=phi, seed=m + k)
        with oz.moduli_table(OPT):
            rc, Ng = oz.required_moduli(dev(A), dev(B), eps)
        terms = planner_terms(A, B)
        lo = required_moduli_from_terms(terms, eps * (1 + 1e-9), table="optimal")
        hi = required_moduli_from_terms(terms, eps * (1 - slack(k)), table="optimal")
        check_between(rc, Ng, lo, hi, 49)


def test_batched_and_noalloc_optimal_table():
    announce("batched and allocation-free calls with the optimal table")
    cases = [(300, 200, 500, 14), (129, 257, 64, 7), (40, 30, 50, 30)]
    As, Bs, Ccm, want = [], [], [], []
    with oz.moduli_table(OPT):
        for q, (m, n, k, N) in enumerate(cases):
            A, B = gemm_inputs(m, n, k, phi=1.0, seed=500 + q)
            As.append(dev(np.ascontiguousarray(A.T)))
            Bs.append(dev(np.ascontiguousarray(B.T)))
            Ccm.append(torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0"))
            want.append(os_ii(A, B, N, table="optimal"))
        oz.gemm_batched_cm(As, Bs, Ccm, [c[:3] for c in cases], [c[3] for c in cases])
        for q, (m, n, k, N) in enumerate(cases):
            assert np.array_equal(host(Ccm[q]).T, want[q]), q
            C = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0")
            rc = oz.ozaki2_gemm_noalloc(64, m, n, k, As[q].data_ptr(), m, Bs[q].data_ptr(), k,
                                        C.data_ptr(), m, N)
            assert rc == oz.OK
            assert np.array_equal(host(C).T, want[q]), q
    # the same batch with the paper's list is a different cached batch
    oz.gemm_batched_cm(As, Bs, Ccm, [c[:3] for c in cases], [c[3] for c in cases])
    assert not np.array_equal(host(Ccm[0]).T, want[0])
    assert oz.ozaki2_sync_status() == oz.OK
