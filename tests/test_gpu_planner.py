"""GPU planner (ozaki2_required_moduli) against the oracle's reading of the
Theorem 1 bound.  The library replaces (|A||B|)_ij by a certified lower bound
(BF16 operands truncated toward zero: at most 2^-6 low; FP32 accumulation of
nonnegative terms: at most k 2^-22 low), so its N lies between the oracle's N
for eps and for eps (1 - slack)."""
import numpy as np
import pytest

from gpu_util import announce, dev
from oracle.bounds import planner_terms, required_moduli_from_terms
from workload import gemm_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402


def slack(k):
    return 2.0 ** -6 + k * 2.0 ** -22 + 1e-9


def effective(rc_or_ok, N, nmax):
    """N, or nmax + 1 when the target is unreachable (rc_or_ok: the oracle's
    reachable flag, or the library's return code)."""
    ok = rc_or_ok if isinstance(rc_or_ok, (bool, np.bool_)) else rc_or_ok == oz.OK
    return N if ok else nmax + 1


def check_between(rc, Ng, lo, hi, nmax):
    g = effective(rc, Ng, nmax)
    a = effective(lo[1], lo[0], nmax)
    b = effective(hi[1], hi[0], nmax)
    assert rc in (oz.OK, oz.ERR_UNREACHABLE)
    assert a <= g <= b, (a, g, b)


@pytest.mark.parametrize("m,n,k,phi,eps", [
    (300, 200, 500, 0.5, 1e-15),
    (300, 200, 500, 4.0, 1e-15),
    (257, 129, 1000, 1.0, 1e-12),
    (64, 700, 256, 2.0, 1e-9),
    (40, 30, 50, 0.0, 1e-15),
    (16, 12, 3 * 2 ** 17, 1.0, 1e-13),     # k beyond 2^17
])
def test_required_moduli_fp64(m, n, k, phi, eps):
    announce(f"planner fp64 m={m} n={n} k={k} phi={phi} eps={eps}")
    A, B = gemm_inputs(m, n, k, phi=phi, seed=m + k)
    rc, Ng = oz.required_moduli(dev(A), dev(B), eps)
    terms = planner_terms(A, B)
    lo = required_moduli_from_terms(terms, eps * (1 + 1e-9))
    hi = required_moduli_from_terms(terms, eps * (1 - slack(k)))
    check_between(rc, Ng, lo, hi, 49)


def test_required_moduli_fp32():
    announce("planner fp32")
    A, B = gemm_inputs(200, 150, 300, phi=1.0, seed=5, dtype=np.float32)
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-6)
    terms = planner_terms(A, B)
    lo = required_moduli_from_terms(terms, 1e-6 * (1 + 1e-9), 32)
    hi = required_moduli_from_terms(terms, 1e-6 * (1 - slack(300)), 32)
    check_between(rc, Ng, lo, hi, 16)


def test_required_moduli_unreachable_and_errors():
    announce("planner unreachable / errors")
    A, B = gemm_inputs(50, 40, 60, seed=2)
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-40)
    assert rc == oz.ERR_UNREACHABLE and Ng == 49
    A[3, 3] = np.inf
    rc, _ = oz.required_moduli(dev(A), dev(B), 1e-15)
    assert rc == oz.ERR_NONFINITE
    rc, _ = oz.required_moduli(dev(A), dev(B), -1.0)
    assert rc == oz.ERR_INVALID_ARG


@pytest.mark.parametrize("phi", [0.0, 1.0, 2.0, 4.0])
def test_required_moduli_4096(phi):
    # The wide-exponent workload (4096^3, phi in {0,1,2,4}) at eps = 1e-15;
    # the oracle's bound ingredients come from FP64 BLAS on the host.
    announce(f"planner 4096^3 phi={phi}")
    A, B = gemm_inputs(4096, 4096, 4096, phi=phi, seed=0)
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-15)
    terms = planner_terms(A, B)
    lo = required_moduli_from_terms(terms, 1e-15 * (1 + 1e-9))
    hi = required_moduli_from_terms(terms, 1e-15 * (1 - slack(4096)))
    print(f"[planner] phi={phi}: oracle {lo[:2]} .. {hi[:2]}, GPU rc={rc} N={Ng}", flush=True)
    check_between(rc, Ng, lo, hi, 49)


def _tiny_product_inputs(e):
    """60 x 70 x 90 inputs in which entry (0, 1) of |A||B| is the single
    product 2^e * 2^e: row 0 of A is [1, 0, 2^e, 0, ...] and column 1 of B
    is [0, 1, 2^e, 0, ...]; everything else is a regular draw."""
    A, B = gemm_inputs(60, 70, 90, phi=0.5, seed=41)
    A[0, :] = 0.0
    A[0, 0], A[0, 2] = 1.0, 2.0 ** e
    B[:, 1] = 0.0
    B[1, 1], B[2, 1] = 1.0, 2.0 ** e
    return A, B


def test_required_moduli_tiny_nonzero_entry():
    # (|A||B|)_01 = 2^-160: positive, but its BF16 / FP32 lower bound
    # underflows to 0.  The entry must still count (the planner's scaling
    # product marks it nonzero): no N is accepted for it, so the GPU answer
    # is UNREACHABLE, at or above the oracle's N (whose FP64 S holds 2^-160).
    announce("planner: nonzero entry whose lower bound of S underflows")
    A, B = _tiny_product_inputs(-80)
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-3)
    lo = required_moduli_from_terms(planner_terms(A, B), 1e-3 * (1 + 1e-9))
    assert rc == oz.ERR_UNREACHABLE and Ng == 49
    assert effective(lo[1], lo[0], 49) <= effective(rc, Ng, 49)
    # 2^-1200 underflows in FP64 too: the oracle agrees that no N works.
    A, B = _tiny_product_inputs(-600)
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-3)
    lo = required_moduli_from_terms(planner_terms(A, B), 1e-3)
    assert not lo[1]
    assert rc == oz.ERR_UNREACHABLE and Ng == 49


def test_required_moduli_exact_zero_entry_is_skipped():
    # A row and a column with disjoint supports give an exactly zero entry,
    # which must not make the target unreachable.
    announce("planner: exactly zero entry")
    A, B = gemm_inputs(60, 70, 90, phi=0.5, seed=42)
    A[0, 45:] = 0.0
    B[:45, 1] = 0.0
    rc, Ng = oz.required_moduli(dev(A), dev(B), 1e-12)
    terms = planner_terms(A, B)
    assert not terms["nz"][0, 1]
    lo = required_moduli_from_terms(terms, 1e-12 * (1 + 1e-9))
    hi = required_moduli_from_terms(terms, 1e-12 * (1 - slack(90)))
    check_between(rc, Ng, lo, hi, 49)
    assert rc == oz.OK


@pytest.mark.parametrize("m,n,k,phi,eps,dt", [
    (120, 90, 200, 0.5, 1e-15, np.complex128),
    (70, 65, 300, 3.0, 1e-15, np.complex128),
    (50, 40, 100, 1.0, 1e-6, np.complex64),
])
def test_complex_required_moduli(m, n, k, phi, eps, dt):
    # ozaki2_zrequired_moduli is the planner on the real embedding on which
    # ozaki2_zgemm runs: its N lies in the oracle's bracket for the embedded
    # matrices (2k terms per entry).
    from oracle.complex_gemm import real_embedding
    from workload import complex_gemm_inputs
    announce(f"complex planner m={m} n={n} k={k} phi={phi} eps={eps}")
    A, B = complex_gemm_inputs(m, n, k, phi=phi, seed=m + n, dtype=dt)
    rc, Ng = oz.required_moduli(dev(A), dev(B), eps)
    Ah, Bh = real_embedding(A, B)
    b = 64 if dt == np.complex128 else 32
    terms = planner_terms(Ah, Bh)
    lo = required_moduli_from_terms(terms, eps * (1 + 1e-9), b)
    hi = required_moduli_from_terms(terms, eps * (1 - slack(2 * k)), b)
    check_between(rc, Ng, lo, hi, 49 if b == 64 else 16)
