"""The C-ABI library loads without a GPU, exports every symbol that
include/ozaki2.h declares, and rejects bad arguments on the host before any
HIP call (so these run on a GPU-less machine)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2602_02549_amd as oz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ozaki2.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ozaki2_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ozaki2_gemm", "ozaki2_sgemm", "ozaki2_required_moduli", "ozaki2_set_stream",
                     "ozaki2_workspace_bytes", "ozaki2_sync_status", "ozaki2_gemm_batched",
                     "ozaki2_debug_stages"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = oz.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []
    out = subprocess.run(["nm", "-D", "--defined-only", oz.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ozaki2_\w+)", out))
    assert set(declared_functions()) <= exported


def test_version_and_workspace_query():
    assert "ozaki2" in oz.ozaki2_version()
    ws = oz.ozaki2_workspace_bytes(64, 8192, 8192, 8192, 14)
    # three INT8 slice sets of N x 8192 x 8192 bytes dominate
    assert ws >= 3 * 14 * 8192 * 8192
    assert oz.ozaki2_workspace_bytes(64, 10, 10, 10, 1) == 0
    assert oz.ozaki2_workspace_bytes(32, 10, 10, 10, 17) == 0     # FP32 allows N <= 16
    assert oz.ozaki2_workspace_bytes(32, 10, 10, 10, 16) > 0
    assert oz.ozaki2_workspace_bytes(64, 10, 10, 1 << 19, 14) == 0
    assert oz.ozaki2_workspace_bytes(64, 10, 10, (1 << 19) - 1, 14) > 0
    assert oz.ozaki2_workspace_bytes(16, 10, 10, 10, 5) == 0
    # m and n stay at or below 2^31 - 256, so that their padding fits in int
    assert oz.ozaki2_workspace_bytes(64, 2 ** 31 - 255, 10, 10, 14) == 0
    assert oz.ozaki2_workspace_bytes(64, 10, 2 ** 31 - 255, 10, 14) == 0
    assert oz.ozaki2_workspace_bytes(64, 2 ** 31 - 256, 10, 10, 14) >= 14 * (2 ** 31 - 256) * 128


FAKE = 0x1000  # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 10), oz.ERR_INVALID_ARG),
    ((4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, 10), oz.ERR_INVALID_ARG),     # lda < m
    ((4, 4, 4, FAKE, 4, FAKE, 3, FAKE, 4, 10), oz.ERR_INVALID_ARG),     # ldb < k
    ((4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 3, 10), oz.ERR_INVALID_ARG),     # ldc < m
    ((4, 4, 4, None, 4, FAKE, 4, FAKE, 4, 10), oz.ERR_INVALID_ARG),     # NULL A
    ((4, 4, 4, FAKE, 4, FAKE, 4, None, 4, 10), oz.ERR_INVALID_ARG),     # NULL C
    ((2 ** 31 - 255, 4, 4, FAKE, 2 ** 31 - 1, FAKE, 4, FAKE, 2 ** 31 - 1, 10), oz.ERR_INVALID_ARG),  # m > 2^31 - 256
    ((4, 2 ** 31 - 255, 4, FAKE, 4, FAKE, 4, FAKE, 4, 10), oz.ERR_INVALID_ARG),  # n > 2^31 - 256
    ((4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1), oz.ERR_N_RANGE),
    ((4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 50), oz.ERR_N_RANGE),
    ((4, 4, 2 ** 19, FAKE, 4, FAKE, 2 ** 19, FAKE, 4, 10), oz.ERR_K_RANGE),      # k >= 2^19
    ((0, 4, 4, None, 1, FAKE, 4, None, 1, 10), oz.OK),                   # m = 0: no-op
    ((4, 0, 4, FAKE, 4, None, 4, None, 4, 10), oz.OK),                   # n = 0: no-op
])
def test_gemm_argument_errors(args, code):
    assert oz.ozaki2_gemm(*args) == code


def test_sgemm_N_limit():
    assert oz.ozaki2_sgemm(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 17) == oz.ERR_N_RANGE
    assert oz.ozaki2_sgemm(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1) == oz.ERR_N_RANGE


def test_batched_rejects_bad_problem_before_running():
    rc = oz.ozaki2_gemm_batched(64, [4, 4, 4, 10, 4, 4, 4, 99], [FAKE, FAKE], [4, 4], [FAKE, FAKE],
                                [4, 4], [FAKE, FAKE], [4, 4])
    assert rc == oz.ERR_N_RANGE
    assert oz.ozaki2_gemm_batched(16, [], [], [], [], [], [], []) == oz.ERR_INVALID_ARG


def test_noalloc_rejections_before_running():
    # The allocation-free entry point checks its arguments and the fixed
    # scratch size on the host; nothing here reaches a device.
    f = oz.ozaki2_gemm_noalloc
    assert f(16, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG
    assert f(64, 4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG
    assert f(64, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 50) == oz.ERR_N_RANGE
    assert f(32, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 17) == oz.ERR_N_RANGE
    assert f(64, 4, 4, 2 ** 19, FAKE, 4, FAKE, 2 ** 19, FAKE, 4, 10) == oz.ERR_K_RANGE
    assert f(64, 0, 4, 4, None, 1, FAKE, 4, None, 1, 10) == oz.OK
    cap = 256 << 20
    # 2048^3 FP64 fits up to N = 21 and not at N = 22; 4096^3 not at N = 14
    # (FP64) or N = 7 (FP32)
    assert oz.ozaki2_workspace_bytes(64, 2048, 2048, 2048, 21) + 256 <= cap
    assert oz.ozaki2_workspace_bytes(64, 2048, 2048, 2048, 22) + 256 > cap
    assert f(64, 2048, 2048, 2048, FAKE, 2048, FAKE, 2048, FAKE, 2048, 22) == oz.ERR_WORKSPACE
    assert oz.ozaki2_workspace_bytes(32, 4096, 4096, 4096, 7) + 256 > cap
    assert f(64, 4096, 4096, 4096, FAKE, 4096, FAKE, 4096, FAKE, 4096, 14) == oz.ERR_WORKSPACE
    assert f(32, 4096, 4096, 4096, FAKE, 4096, FAKE, 4096, FAKE, 4096, 7) == oz.ERR_WORKSPACE


def test_complex_argument_errors_and_workspace():
    # Host-side checks of ozaki2_zgemm / ozaki2_cgemm (nothing reaches a device).
    z, c, q = oz.ozaki2_zgemm, oz.ozaki2_cgemm, oz.ozaki2_complex_workspace_bytes
    assert z(4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG     # lda < m
    assert z(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 2 ** 30, 10) == oz.ERR_INVALID_ARG  # ldc >= 2^30
    assert z(4, 4, 4, None, 4, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG
    assert z(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 50) == oz.ERR_N_RANGE
    assert c(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 17) == oz.ERR_N_RANGE
    assert z(4, 4, 2 ** 18, FAKE, 4, FAKE, 2 ** 18, FAKE, 4, 10) == oz.ERR_K_RANGE  # 2k >= 2^19
    assert z(0, 4, 4, None, 1, FAKE, 4, None, 1, 10) == oz.OK
    # the embedded real problem, formed in place by the slice kernels, is
    # 2m x n x 2k with its k halves 128-aligned (here 2 x 256): the workspace
    # is that problem's, at least the real 600 x 200 x 500 one's
    real = oz.ozaki2_workspace_bytes(64, 600, 200, 500, 14)
    got = q(64, 300, 200, 250, 14)
    assert got >= oz.ozaki2_workspace_bytes(64, 600, 200, 512, 14) >= real
    # both forms read the complex inputs in place: no element-size-dependent copies
    assert q(32, 300, 200, 250, 14) == got
    # k >= 2^18 is served by the 3-product form only; k >= 2^19 by neither
    assert q(64, 300, 200, 2 ** 19, 14) == 0 and q(64, 300, 200, 2 ** 19 - 1, 14) > 0
    assert q(64, 300, 200, 2 ** 18, 14) > 0
    assert q(32, 300, 200, 250, 17) == 0 and q(64, 0, 4, 4, 14) == 0


def test_complex3m_argument_errors_and_workspace():
    # Host-side checks of ozaki2_zgemm3m / ozaki2_cgemm3m (nothing reaches a device).
    z, c, q = oz.ozaki2_zgemm3m, oz.ozaki2_cgemm3m, oz.ozaki2_complex_workspace_bytes
    assert z(4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG     # lda < m
    assert z(4, 4, 4, FAKE, 4, FAKE, 3, FAKE, 4, 10) == oz.ERR_INVALID_ARG     # ldb < k
    assert z(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 3, 10) == oz.ERR_INVALID_ARG     # ldc < m
    assert z(4, 4, 4, FAKE, 4, None, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG
    assert z(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1) == oz.ERR_N_RANGE
    assert c(4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 17) == oz.ERR_N_RANGE
    assert z(4, 4, 2 ** 19, FAKE, 4, FAKE, 2 ** 19, FAKE, 4, 10) == oz.ERR_K_RANGE
    assert c(-1, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 10) == oz.ERR_INVALID_ARG
    assert z(4, 0, 4, FAKE, 4, None, 4, None, 4, 10) == oz.OK
    # 3 INT32 product planes per modulus instead of the embedded 2m x n
    # plane; the query covers both forms
    four = q(64, 300, 200, 250, 14)
    assert four > 0 and q(64, 300, 200, 2 ** 18 + 5, 14) > four


def test_debug_and_log2f_argument_errors():
    assert oz.ozaki2_debug_log2f(None, None, 0) == oz.OK
    assert oz.ozaki2_debug_log2f(None, None, 5) == oz.ERR_INVALID_ARG
    assert oz.ozaki2_debug_stages(64, 4, 4, 4, FAKE, 4, FAKE, 4, 10, [None] * 11) == oz.ERR_INVALID_ARG
    outs = [None] * 9 + [FAKE]
    assert oz.ozaki2_debug_stages(64, 4, 4, 4, FAKE, 4, FAKE, 4, 10, outs[:9]) == oz.ERR_INVALID_ARG
    assert oz.ozaki2_debug_stages(64, 4, 4, 4, FAKE, 4, FAKE, 4, 10, outs + [None] * 7) == oz.ERR_INVALID_ARG
    assert oz.ozaki2_debug_stages(64, 4, 4, 4, FAKE, 4, FAKE, 4, 50, outs + [None] * 6) == oz.ERR_N_RANGE


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(oz, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(oz, "_lib", None)
    with pytest.raises(RuntimeError):
        oz.lib()


def test_batched_workspace_query():
    # Degenerate problems need no workspace; each active problem adds its own
    # layout; invalid arguments give 0.  (No device work is involved.)
    q = oz.ozaki2_batched_workspace_bytes
    assert q(64, []) == 0
    assert q(64, [5, 4, 0, 10, 0, 7, 9, 12]) == 0
    one = q(64, [300, 200, 500, 14])
    two = q(64, [300, 200, 500, 14, 100, 90, 300, 20])
    assert 0 < one < two
    assert q(64, [300, 200, 500, 14, 5, 4, 0, 10]) == one
    assert q(64, [300, 200, 500, 50]) == 0          # N out of range
    assert q(32, [300, 200, 500, 17]) == 0          # FP32 allows N <= 16
    assert q(64, [300, 200, 1 << 19, 14]) == 0
    assert q(64, [300, 200, (1 << 17) + 1, 14]) > 0
    assert q(16, [300, 200, 500, 14]) == 0
    # at least the moduli slices and W of every active problem
    assert two >= 20 * (128 * 384 + 128 * 384 + 128 * 128) + 14 * (384 * 512 + 256 * 512 + 256 * 384)


def test_certified_argument_errors_and_workspace_query():
    # Host-side validation of ozaki2_gemm_certified (nothing reaches the device).
    c = oz.ozaki2_gemm_certified
    assert c(16, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1e-14, 0)[0] == oz.ERR_INVALID_ARG
    assert c(64, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 0.0, 0)[0] == oz.ERR_INVALID_ARG
    assert c(64, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, float("nan"), 0)[0] == oz.ERR_INVALID_ARG
    assert c(64, 4, 4, 4, FAKE, 3, FAKE, 4, FAKE, 4, 1e-14, 0)[0] == oz.ERR_INVALID_ARG   # lda < m
    assert c(64, 4, 4, 4, FAKE, 4, FAKE, 4, None, 4, 1e-14, 0)[0] == oz.ERR_INVALID_ARG   # NULL C
    assert c(64, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1e-14, 1)[0] == oz.ERR_N_RANGE
    assert c(32, 4, 4, 4, FAKE, 4, FAKE, 4, FAKE, 4, 1e-6, 17)[0] == oz.ERR_N_RANGE
    assert c(64, 4, 4, 2 ** 19, FAKE, 4, FAKE, 2 ** 19, FAKE, 4, 1e-14, 0)[0] == oz.ERR_K_RANGE
    assert c(64, 0, 4, 4, None, 1, FAKE, 4, None, 1, 1e-14, 0) == (oz.OK, 2, 0.0)   # m = 0: no-op
    q = oz.ozaki2_certified_workspace_bytes
    assert q(64, 300, 200, 500, 14) > oz.ozaki2_workspace_bytes(64, 300, 200, 500, 14)
    assert q(64, 300, 200, 500, 20) > q(64, 300, 200, 500, 14)
    assert q(64, 300, 200, 500, 50) == 0 and q(32, 300, 200, 500, 17) == 0 and q(64, 0, 4, 4, 14) == 0


def test_tuning_knobs():
    # Set, read back through `previous`, restore; bad knobs and values rejected.
    t = oz.ozaki2_debug_tuning
    rc, prev = t(oz.KNOB_SLICE_WORKGROUPS, 5)
    assert rc == oz.OK and prev == 0
    assert t(oz.KNOB_SLICE_WORKGROUPS, 0) == (oz.OK, 5)
    assert t(oz.KNOB_GEMM_TILE, 3)[0] == oz.ERR_INVALID_ARG
    assert t(oz.KNOB_BATCH_SPLIT, -2)[0] == oz.ERR_INVALID_ARG
    assert t(oz.KNOB_BATCH_GRAPH, 2)[0] == oz.ERR_INVALID_ARG
    assert t(oz.KNOB_BATCH_PERSIST, 3)[0] == oz.ERR_INVALID_ARG
    with oz.tuning(oz.KNOB_BATCH_PERSIST, 2):
        assert t(oz.KNOB_BATCH_PERSIST, 2) == (oz.OK, 2)
    assert t(99, 0)[0] == oz.ERR_INVALID_ARG
    with oz.tuning(oz.KNOB_BATCH_SPLIT, 4):
        assert t(oz.KNOB_BATCH_SPLIT, 4) == (oz.OK, 4)
    assert t(oz.KNOB_BATCH_SPLIT, -1) == (oz.OK, -1)


def test_split_k_scratch_in_workspace():
    # A small output with long k splits its products: the workspace holds the
    # partial results.  64 x 64 x 262144, N = 14 (one 128 x 128 tile, 2048
    # groups of 128 k): the residue products split 512 / 14 = 36 ways (36 x 14
    # partial planes of 128 x 128 bytes), the scaling product 16 ways (INT32,
    # a smaller region).  With split-k off the region is absent.
    q = oz.ozaki2_workspace_bytes
    shapes = [(64, 64, 262144, 14), (4096, 4096, 4096, 14)]
    with_split = [q(64, *s) for s in shapes]
    rc, prev = oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, 1)
    assert rc == oz.OK
    try:
        without = [q(64, *s) for s in shapes]
    finally:
        oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, prev)
    assert with_split[0] - without[0] == 36 * 14 * 128 * 128
    # an output that fills the GPU does not split: no region
    assert with_split[1] == without[1]
    assert oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, 7)[0] == oz.ERR_INVALID_ARG


def test_batched_split_k_scratch():
    # A batch of at most 64 active problems holds each long-k problem's
    # split-k scratch (the same region as the single call's) for the
    # per-problem form; a larger batch holds none.
    q = oz.ozaki2_batched_workspace_bytes
    shape = [64, 64, 262144, 14]
    one = q(64, shape)
    rc, prev = oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, 1)
    assert rc == oz.OK
    try:
        one_plain = q(64, shape)
    finally:
        oz.ozaki2_debug_tuning(oz.KNOB_SPLIT_K, prev)
    assert one - one_plain == 36 * 14 * 128 * 128
    assert q(64, shape * 64) == 64 * one
    assert q(64, shape * 65) == 65 * one_plain
    # degenerate problems do not count towards the 64
    assert q(64, shape * 64 + [5, 4, 0, 10]) == 64 * one


def test_complex_planner_argument_errors():
    # Host-side checks of ozaki2_zrequired_moduli (nothing reaches a device).
    f = oz.ozaki2_zrequired_moduli
    assert f(16, 4, 4, 4, FAKE, 4, FAKE, 4, 1e-15)[0] == oz.ERR_INVALID_ARG
    assert f(64, 4, 4, 4, FAKE, 4, FAKE, 4, 0.0)[0] == oz.ERR_INVALID_ARG
    assert f(64, 4, 4, 4, FAKE, 3, FAKE, 4, 1e-15)[0] == oz.ERR_INVALID_ARG     # lda < m
    assert f(64, 4, 4, 4, None, 4, FAKE, 4, 1e-15)[0] == oz.ERR_INVALID_ARG
    assert f(64, 4, 4, 2 ** 18, FAKE, 4, FAKE, 2 ** 18, 1e-15)[0] == oz.ERR_K_RANGE
    assert f(32, 0, 4, 4, None, 1, FAKE, 4, 1e-6) == (oz.OK, 2)


def test_mfma_probe_argument_errors():
    assert oz.ozaki2_debug_mfma_probe(0)[0] == oz.ERR_INVALID_ARG
    assert oz.ozaki2_debug_mfma_probe(2 ** 20 + 1)[0] == oz.ERR_INVALID_ARG
    assert oz.ozaki2_debug_mfma_probe(16, 2)[0] == oz.ERR_INVALID_ARG
