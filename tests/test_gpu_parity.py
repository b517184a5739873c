"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer stages (mu', nu', Cbar maxima, mu, nu, A'_l, B'_l, the INT32 products
C'_l, W_l) must be bit-exact, and so must the FP64 intermediates C'(1), C'(2),
Q and C'' of Algorithm 3; log2f must equal the correctly rounded value on every input;
outputs must be within 2^-50 (FP64) / 2^-22 (FP32) of the oracle per entry.
The library follows the oracle's operation order in the CRT (explicit fma,
fixed l order), so the outputs are in fact required to be bit-identical too.
"""
import numpy as np
import pytest

from gpu_util import announce, compare_stages, dev, host, rel_close
from oracle.ozaki2 import log2f_many, os_ii
from workload import gemm_inputs, wrap_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402

REL64 = 2.0 ** -50
REL32 = 2.0 ** -22


def run_stage_case(m, n, k, N, phi, seed, dtype):
    announce(f"stages m={m} n={n} k={k} N={N} phi={phi} seed={seed} {np.dtype(dtype).name}")
    A, B = gemm_inputs(m, n, k, phi=phi, seed=seed, dtype=dtype)
    got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), N).items()}
    C_ref, st = os_ii(A, B, N, stages=True)
    bad = compare_stages(got, st, C_ref, N)
    assert bad == [], bad
    tol = REL64 if dtype == np.float64 else REL32
    assert np.all(rel_close(got["CT"].T, C_ref, tol))
    assert oz.ozaki2_sync_status() == oz.OK


def test_stages_config_256():
    # The small FP64 configuration exactly (256^3, N = 14, phi = 0.5, seed 0):
    # every stage bit-exact, plus the exact big-integer product A'B' against
    # the CRT reconstruction of the GPU's W_l.
    announce("stages 256^3 N=14 phi=0.5 seed=0")
    A, B = gemm_inputs(256, 256, 256, phi=0.5, seed=0)
    got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), 14).items()}
    C_ref, st = os_ii(A, B, 14, stages=True)
    assert compare_stages(got, st, C_ref, 14) == []
    assert "ClT" in got and "CppT" in got
    from oracle.constants import constants
    from oracle.exact import exact_int_product
    const = constants(14, 64)
    ApBp = exact_int_product(st["Ap"], st["Bp"])
    P = int(const.P)
    recon = np.zeros((256, 256), dtype=object)
    for l in range(14):
        recon = recon + np.asarray(got["WT"][l].T, dtype=object) * int(const.x[l])
    recon = np.vectorize(lambda v: ((int(v) + P // 2) % P) - P // 2, otypes=[object])(recon)
    assert np.array_equal(recon, ApBp)
    assert oz.ozaki2_sync_status() == oz.OK


def test_int32_wrap_at_k_max():
    # k = 2^17 with every residue modulo 256 equal to -128 (N = 14): the
    # p = 256 residue product sums k terms of 2^14 to 2^31, which the INT8
    # matrix cores must wrap to -2^31 (W = 0), not saturate (W = -1).  Every
    # stage bit-exact against the oracle (128x128 kernel).  Then a 512 x 512
    # problem of the same kind through the single call (128x128 tiles) and
    # the batched path with all 256x256 and all 128x128 tiles: bit-identical,
    # and equal to the oracle on sampled entries.
    m, n, k, N = 40, 33, 2 ** 17, 14
    announce(f"int32 wrap m={m} n={n} k={k} N={N}")
    A, B = wrap_inputs(m, n, k, seed=2)
    got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), N).items()}
    C_ref, st = os_ii(A, B, N, stages=True)
    l = list(st["const"].p).index(256)
    assert np.all(st["Cl"][l] == -2 ** 31)
    assert np.all(got["ClT"][l] == -2 ** 31)      # the wrap, seen on the matrix cores
    assert np.all(got["WT"][l] == 0)
    bad = compare_stages(got, st, C_ref, N)
    assert bad == [], bad
    assert oz.ozaki2_sync_status() == oz.OK
    assert np.array_equal(host(oz.gemm(dev(A), dev(B), N)), C_ref)

    m = n = 512
    announce(f"int32 wrap m={m} n={n} k={k} N={N} single and batched")
    A, B = wrap_inputs(m, n, k, seed=3)
    ref = host(oz.gemm(dev(A), dev(B), N))
    rows, cols = np.array([0, 77, 300, 511]), np.array([3, 128, 255, 500])
    want, st = os_ii(A, B, N, rows=rows, cols=cols, stages=True)
    assert np.all(st["Cl"][l] == -2 ** 31)
    assert np.array_equal(ref[np.ix_(rows, cols)], want)
    dA, dB = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    del A, B
    for split in (0, 1000000):
        announce(f"int32 wrap batched split={split}")
        with oz.tuning(oz.KNOB_BATCH_SPLIT, split):
            Cc = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0")
            oz.gemm_batched_cm([dA], [dB], [Cc], [(m, n, k)], [N])
        assert oz.ozaki2_sync_status() == oz.OK
        assert np.array_equal(host(Cc).T, ref), f"split {split}"


@pytest.mark.parametrize("k", [2 ** 17 + 1, 3 * 2 ** 17])
def test_k_beyond_2_17(k):
    # k above the paper's 2^17 (up to 2^19 - 1): Cbar maxima above 2^29,
    # residue products reduced mod p_l every 2^17 of k.  Every stage
    # bit-exact (C'_l congruent mod p_l), through the single call and a batch.
    m, n, N = 16, 12, 14
    announce(f"k beyond 2^17: m={m} n={n} k={k} N={N}")
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=k % 997)
    run_stage_case(m, n, k, N, 1.0, seed=k % 997, dtype=np.float64)
    ref = host(oz.gemm(dev(A), dev(B), N))
    cases = [(A, B, N), gemm_inputs(30, 20, 100, phi=1.0, seed=5) + (13,)]
    Cb = oz.gemm_batched([dev(a) for a, _, _ in cases], [dev(b) for _, b, _ in cases],
                         [c[2] for c in cases])
    assert np.array_equal(host(Cb[0]), ref)
    assert np.array_equal(host(Cb[1]), os_ii(cases[1][0], cases[1][1], 13))
    assert oz.ozaki2_sync_status() == oz.OK


def test_k_beyond_2_17_residue_product_past_int32():
    # Every term of the p = 255 residue product is 127^2 (fold-stressing
    # inputs), so at k = 2^18 the product 2^18 127^2 exceeds 2^31: without
    # the reduction every 2^17 of k the INT32 accumulator would wrap and W
    # would be off by one modulo 255.  Every stage bit-exact against the
    # oracle, the accumulator within INT32 and congruent to the product.
    from pins import fold_inputs
    m, n, k, N = 16, 8, 2 ** 18, 14
    announce(f"fold-stressing inputs m={m} n={n} k={k} N={N}")
    A, B = fold_inputs(m, n, k, N)
    got = {kk: host(v) for kk, v in oz.debug_stages(dev(A), dev(B), N).items()}
    C_ref, st = os_ii(A, B, N, stages=True)
    l = list(st["const"].p).index(255)
    assert np.all(np.abs(st["Cl"][l]) == k * 127 * 127)
    assert compare_stages(got, st, C_ref, N) == []
    assert oz.ozaki2_sync_status() == oz.OK


def test_single_call_256_tiles_ragged():
    # 768 x 1000, k = 130, N = 16: padding n to 256 costs nothing over 128,
    # and the 16 residue products have 3 x 4 x 16 = 192 tiles of 256 x 256,
    # so the single call takes the 256 x 256 kernel for them (the scaling
    # product, 12 tiles, the 128 x 128 one).  The result has the bits of the
    # batched path with all tiles 128 x 128, and the oracle's on sampled
    # entries.
    m, n, k, N = 768, 1000, 130, 16
    announce(f"single call, 256x256 residue tiles, m={m} n={n} k={k} N={N}")
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=11)
    C = host(oz.gemm(dev(A), dev(B), N))
    assert oz.ozaki2_sync_status() == oz.OK
    rows, cols = np.array([0, 255, 256, 511, 767]), np.array([0, 255, 256, 767, 768, 999])
    assert np.array_equal(C[np.ix_(rows, cols)], os_ii(A, B, N, rows=rows, cols=cols))
    dA, dB = dev(np.ascontiguousarray(A.T)), dev(np.ascontiguousarray(B.T))
    Cc = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0")
    with oz.tuning(oz.KNOB_BATCH_SPLIT, 1000000):
        oz.gemm_batched_cm([dA], [dB], [Cc], [(m, n, k)], [N])
    assert oz.ozaki2_sync_status() == oz.OK
    assert np.array_equal(host(Cc).T, C)


def test_stages_256_tiles():
    # 768 x 1000 x 130, N = 16: the residue products run on the 256 x 256
    # kernel (192 tiles of 256 x 256 over the 16 products, and padding n to
    # 256 costs nothing over 128).  Every stage bit-exact, the INT32 products
    # C'_l and the full W_l of that kernel included.
    m, n, k, N = 768, 1000, 130, 16
    assert (m // 256) * ((n + 255) // 256) * N > 128
    run_stage_case(m, n, k, N, 1.0, seed=31, dtype=np.float64)


@pytest.mark.parametrize("m,n,k,N,phi", [
    (300, 200, 500, 14, 0.5),     # several 128-tiles in each direction, ragged tails
    (64, 64, 64, 2, 0.5),
    (1, 1, 1, 7, 0.5),
    (257, 129, 130, 20, 1.0),
    (100, 90, 300, 49, 2.0),
    (33, 300, 129, 11, 4.0),
    # residue paths at the ends of their N ranges: two limbs (N = 12..22),
    # three limbs (N = 23..31), three exact steps (N = 32..40), four (from 41)
    (70, 65, 200, 12, 1.0),
    (70, 65, 200, 15, 1.0),
    (70, 65, 200, 22, 2.0),
    (70, 65, 200, 23, 2.0),
    (70, 65, 200, 24, 3.0),
    (70, 65, 200, 30, 4.0),
    (70, 65, 200, 31, 4.0),
    (70, 65, 200, 32, 4.0),
    (70, 65, 200, 40, 4.0),
    (70, 65, 200, 41, 4.0),
    # the fused column abs-max and Bbar kernel: a wave per column up to
    # k_pad = 2048, a workgroup per column above (ragged k), two passes
    # beyond 8192
    (33, 70, 2048, 7, 0.5),
    (33, 70, 2049, 7, 0.5),
    (40, 33, 3001, 14, 1.0),
    (20, 17, 8300, 9, 1.0),
])
def test_stages_fp64(m, n, k, N, phi):
    run_stage_case(m, n, k, N, phi, seed=m + n + k + N, dtype=np.float64)


@pytest.mark.parametrize("m,n,k,N,phi", [
    (300, 200, 500, 7, 0.5),
    (130, 70, 260, 2, 1.0),
    (64, 257, 100, 16, 0.5),
    (40, 33, 3001, 7, 1.0),
])
def test_stages_fp32(m, n, k, N, phi):
    run_stage_case(m, n, k, N, phi, seed=m + n + k + N, dtype=np.float32)


@pytest.mark.parametrize("cap", ["1", "5"])
def test_slices_few_workgroups(cap):
    # The slice kernels walk their tiles in a grid-stride loop, prefetching the
    # next tile.  Capped at `cap` workgroups, every workgroup walks many tiles
    # (with 5, unevenly many).  Every stage stays bit-exact on each residue
    # path (2 and 3 limbs, one, three and four exact steps, FP32), and the
    # grouped kernels of a batch give the oracle's result.
    with oz.tuning(oz.KNOB_SLICE_WORKGROUPS, int(cap)):
        _slices_few_workgroups(cap)


def _slices_few_workgroups(cap):
    for m, n, k, N, phi, dt in [(300, 200, 500, 14, 0.5, np.float64), (257, 129, 130, 16, 1.0, np.float64),
                                (100, 90, 300, 7, 2.0, np.float64), (90, 70, 150, 28, 3.0, np.float64),
                                (60, 50, 100, 36, 4.0, np.float64), (70, 65, 200, 49, 4.0, np.float64),
                                (130, 70, 260, 7, 1.0, np.float32)]:
        run_stage_case(m, n, k, N, phi, seed=int(cap) + m + N, dtype=dt)
    announce(f"batched with {cap} slice workgroups")
    cases = [(300, 200, 500, 14), (129, 257, 64, 16), (40, 30, 50, 30), (33, 20, 40, 36)]
    As, Bs, Ccm = [], [], []
    for q, (m, n, k, N) in enumerate(cases):
        A, B = gemm_inputs(m, n, k, phi=1.0, seed=900 + q)
        As.append(A)
        Bs.append(B)
        Ccm.append(torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0"))
    oz.gemm_batched_cm([dev(np.ascontiguousarray(A.T)) for A in As],
                       [dev(np.ascontiguousarray(B.T)) for B in Bs], Ccm,
                       [(m, n, k) for m, n, k, _ in cases], [c[3] for c in cases])
    assert oz.ozaki2_sync_status() == oz.OK
    for q, (A, B, (m, n, k, N)) in enumerate(zip(As, Bs, cases)):
        assert np.array_equal(host(Ccm[q]).T, os_ii(A, B, N)), f"batched problem {q}"


def test_gemm_captured_in_a_graph():
    # ozaki2_gemm enqueues kernels only (no memset or copy nodes), so once the
    # workspace has grown a caller can capture it.  The graph is replayed three
    # times with other library work, synchronisation and a reset of C between
    # the replays; every replay must give the eager call's bits.
    announce("ozaki2_gemm captured in a graph")
    m, n, k, N = 300, 200, 500, 14
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=21)
    ref = host(oz.gemm(dev(A), dev(B), N))          # grows the workspace
    dA = dev(np.ascontiguousarray(A.T))
    dB = dev(np.ascontiguousarray(B.T))
    C = torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc = oz.ozaki2_gemm(m, n, k, dA.data_ptr(), m, dB.data_ptr(), k, C.data_ptr(), m, N)
    assert rc == oz.OK
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(C).T, ref), f"replay {rep}"
        X, Y = gemm_inputs(120, 90, 150, seed=30 + rep)
        assert np.array_equal(host(oz.gemm(dev(X), dev(Y), 12)), os_ii(X, Y, 12))
    assert oz.ozaki2_sync_status() == oz.OK


def test_leading_dimensions_and_views():
    # lda > m, ldb > k, ldc > m through the raw C ABI (submatrices of bigger buffers).
    announce("leading dimensions m=90 n=70 k=110 N=13")
    m, n, k, N = 90, 70, 110, 13
    A, B = gemm_inputs(m, n, k, phi=1.0, seed=3)
    lda, ldb, ldc = m + 7, k + 5, m + 3
    Abuf = np.full((k, lda), np.nan)
    Abuf[:, :m] = A.T
    Bbuf = np.full((n, ldb), np.nan)
    Bbuf[:, :k] = B.T
    dA, dB = dev(Abuf), dev(Bbuf)
    dC = torch.full((n, ldc), 7.0, dtype=torch.float64, device="cuda:0")
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    rc = oz.ozaki2_gemm(m, n, k, dA.data_ptr(), lda, dB.data_ptr(), ldb, dC.data_ptr(), ldc, N)
    assert rc == oz.OK
    Cbuf = host(dC)
    assert np.all(Cbuf[:, m:] == 7.0)          # untouched padding of C
    assert np.array_equal(Cbuf[:, :m].T, os_ii(A, B, N))
    assert oz.ozaki2_sync_status() == oz.OK


def test_edge_cases():
    announce("edge cases: k=0, zero rows/columns, integer inputs")
    # k = 0: C = 0
    C = oz.gemm(torch.zeros((5, 0), dtype=torch.float64, device="cuda:0"),
                torch.zeros((0, 4), dtype=torch.float64, device="cuda:0"), 10)
    assert torch.all(C == 0).item()
    # zero rows / columns give exact zeros, everything else matches the oracle
    A, B = gemm_inputs(70, 60, 90, phi=1.0, seed=8)
    A[5, :] = 0.0
    B[:, 9] = 0.0
    got = host(oz.gemm(dev(A), dev(B), 15))
    assert np.all(got[5, :] == 0) and np.all(got[:, 9] == 0)
    assert np.array_equal(got, os_ii(A, B, 15))
    # integer inputs with no truncation reproduce AB exactly
    rng = np.random.default_rng(4)
    Ai = rng.integers(-20, 21, (40, 30)).astype(np.float64)
    Bi = rng.integers(-20, 21, (30, 20)).astype(np.float64)
    assert np.array_equal(host(oz.gemm(dev(Ai), dev(Bi), 5)), Ai @ Bi)
    # subnormal and huge magnitudes in one matrix
    A, B = gemm_inputs(40, 40, 64, phi=0.5, seed=9)
    A[3, :] *= 2.0 ** -1060          # a subnormal row
    A[4, 7] = 1e300                   # one huge entry (products stay finite)
    B[:, 2] *= 2.0 ** -900            # a tiny column
    assert np.array_equal(host(oz.gemm(dev(A), dev(B), 18)), os_ii(A, B, 18))
    assert oz.ozaki2_sync_status() == oz.OK


def test_nonfinite_input_sets_status_and_nan():
    announce("non-finite input")
    A, B = gemm_inputs(40, 30, 50, seed=2)
    A[3, 4] = np.nan
    got = host(oz.gemm(dev(A), dev(B), 10))
    assert np.all(np.isnan(got))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert oz.ozaki2_sync_status() == oz.OK          # cleared by the read
    B[1, 1] = np.inf
    A[3, 4] = 1.0
    assert np.all(np.isnan(host(oz.gemm(dev(A), dev(B), 10))))
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE


def test_deterministic():
    announce("determinism 512x384x700 N=16")
    A, B = gemm_inputs(512, 384, 700, phi=2.0, seed=12)
    dA, dB = dev(A), dev(B)
    c1 = host(oz.gemm(dA, dB, 16))
    c2 = host(oz.gemm(dA, dB, 16))
    assert np.array_equal(c1, c2)


def test_log2f_exhaustive():
    # Every integer-valued FP32 number in [1, 2^29] (the domain of Dbar).
    announce("log2f exhaustive over integer-valued FP32 in [1, 2^29]")
    parts = [np.arange(1, 2 ** 24 + 1, dtype=np.float64)]
    for s in range(1, 6):
        parts.append(np.arange(2 ** (23 + s) + 2 ** s, 2 ** (24 + s) + 1, 2 ** s, dtype=np.float64))
    d = np.concatenate(parts).astype(np.float32)
    assert np.all(d.astype(np.float64) == np.concatenate(parts))
    dd = dev(d)
    out = torch.empty_like(dd)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    assert oz.ozaki2_debug_log2f(dd.data_ptr(), out.data_ptr(), d.size) == oz.OK
    got = host(out)
    chunk = 1 << 23
    for s in range(0, d.size, chunk):
        ref = log2f_many(d[s:s + chunk])
        assert np.array_equal(got[s:s + chunk], ref), f"log2f mismatch in chunk at {s}"


@pytest.mark.parametrize("dtype,N,size", [(np.float64, 14, 8192), (np.float32, 7, 8192),
                                          (np.float32, 7, 16384)])
def test_full_size_sampled(dtype, N, size):
    # The bench workload (FP64 8192^3) in the launch configuration the
    # benchmark times, and the FP32 16384^3 emulated SGEMM; sampled rows x
    # columns against the oracle, which needs only those rows/columns of the
    # scaled integers plus full-matrix row/column maxima of Cbar.
    m = n = k = size
    announce(f"full size {m}^3 N={N} {np.dtype(dtype).name}")
    A, B = gemm_inputs(m, n, k, phi=0.5, seed=0, dtype=dtype)
    got = host(oz.gemm(dev(A), dev(B), N))
    rng = np.random.default_rng(99)
    rows = np.sort(rng.choice(m, 12, replace=False))
    cols = np.sort(rng.choice(n, 12, replace=False))
    rows[-1], cols[-1] = m - 1, n - 1
    ref = os_ii(A, B, N, rows=rows, cols=cols)
    sub = got[np.ix_(rows, cols)]
    assert np.array_equal(sub, ref)
    assert oz.ozaki2_sync_status() == oz.OK


@pytest.mark.parametrize("phi", [0.0, 1.0, 2.0, 4.0])
def test_wide_exponent_4096_sampled(phi):
    # The wide-exponent workload at 4096^3 with N from the bound at 1e-15
    # (49 where it is unreachable): sampled rows x columns against the oracle.
    n = 4096
    A, B = gemm_inputs(n, n, n, phi=phi, seed=0)
    dA, dB = dev(A), dev(B)
    rc, N = oz.required_moduli(dA, dB, 1e-15)
    assert rc in (oz.OK, oz.ERR_UNREACHABLE)
    announce(f"wide exponent 4096^3 phi={phi} N={N}")
    got = host(oz.gemm(dA, dB, N))
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n, 10, replace=False))
    cols = np.sort(rng.choice(n, 10, replace=False))
    rows[0], cols[-1] = 0, n - 1
    assert np.array_equal(got[np.ix_(rows, cols)], os_ii(A, B, N, rows=rows, cols=cols))
    assert oz.ozaki2_sync_status() == oz.OK


@pytest.mark.parametrize("phi,N", [(0.5, 14), (4.0, 30)])
def test_error_within_theorem1_bound_4096(phi, N):
    # Theorem 1 on the GPU's own output at 4096^3, on sampled entries:
    # |AB - C| <= est1 <= est2 with the exact AB and the exact A'B'.
    from oracle.bounds import theorem1
    from oracle.exact import abs_error, exact_int_product, exact_product
    n = 4096
    announce(f"Theorem 1 on GPU output 4096^3 phi={phi} N={N}")
    A, B = gemm_inputs(n, n, n, phi=phi, seed=3)
    got = host(oz.gemm(dev(A), dev(B), N))
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, 8, replace=False))
    cols = np.sort(rng.choice(n, 8, replace=False))
    C_ref, st = os_ii(A, B, N, rows=rows, cols=cols, stages=True)
    sub = got[np.ix_(rows, cols)]
    assert np.array_equal(sub, C_ref)
    ApBp = exact_int_product(st["Ap"], st["Bp"])
    est1, est2 = theorem1(A, B, st, ApBp)
    err = abs_error(sub, exact_product(A, B, rows, cols))
    for idx in np.ndindex(err.shape):
        assert err[idx] <= float(est1[idx]) <= float(est2[idx]), idx
    assert oz.ozaki2_sync_status() == oz.OK
