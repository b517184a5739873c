"""GPU parity of the batched entry point (ozaki2_gemm_batched).

Every problem of a batch must give exactly the single-problem result, which
the parity tests pin bit-exactly to the oracle; small problems are also
checked against the oracle directly, and the full uneven 512-problem workload
on sampled outputs.  The batch runs as one captured graph, so replays are
checked with other eager work on the same stream between them.
"""
import numpy as np
import pytest

from gpu_util import announce, dev, host
from oracle.ozaki2 import os_ii
from workload import batched_inputs, gemm_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2602_02549_amd as oz  # noqa: E402

# (m, n, k, N): ragged tails, tiny and degenerate sizes, N from 2 to 49, and
# problems large enough for the 256x256 kernel.
SMALL = [
    (300, 200, 500, 14), (1, 1, 1, 7), (64, 64, 64, 2), (257, 129, 130, 20), (100, 90, 300, 49),
    (33, 300, 129, 11), (5, 4, 0, 10), (0, 7, 9, 12), (6, 0, 9, 12), (513, 770, 260, 16),
    (1024, 1024, 128, 13), (70, 60, 90, 15),
]


def make_batch(cases, dtype, seed):
    As, Bs = [], []
    for q, (m, n, k, N) in enumerate(cases):
        A, B = gemm_inputs(m, n, k, phi=1.0, seed=seed + q, dtype=dtype)
        As.append(A)
        Bs.append(B)
    return As, Bs


def cm(X):
    """Column-major device copy of X (a (cols x rows) contiguous tensor)."""
    return dev(np.ascontiguousarray(X.T))


def run_batched(As, Bs, Ns, fill=np.nan):
    shapes = [(A.shape[0], B.shape[1], A.shape[1]) for A, B in zip(As, Bs)]
    Acm = [cm(A) for A in As]
    Bcm = [cm(B) for B in Bs]
    Ccm = [torch.full((n, m), fill, dtype=Acm[0].dtype, device="cuda:0") for (m, n, _) in shapes]
    oz.gemm_batched_cm(Acm, Bcm, Ccm, shapes, Ns)
    return Acm, Bcm, Ccm, shapes


def single(A, B, N):
    return host(oz.gemm(dev(A), dev(B), N))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_matches_single_and_oracle(dtype):
    cases = [(m, n, k, min(N, 16) if dtype == np.float32 else N) for m, n, k, N in SMALL]
    announce(f"batched {len(cases)} problems {np.dtype(dtype).name}")
    As, Bs = make_batch(cases, dtype, seed=100)
    Ns = [c[3] for c in cases]
    _, _, Ccm, _ = run_batched(As, Bs, Ns)
    assert oz.ozaki2_sync_status() == oz.OK
    for q, (A, B, N) in enumerate(zip(As, Bs, Ns)):
        got = host(Ccm[q]).T
        ref = single(A, B, N)
        assert np.array_equal(got, ref), f"problem {q} {cases[q]}"
        if A.shape[0] * B.shape[1] * max(A.shape[1], 1) <= 300 * 300 * 500:
            assert np.array_equal(got, os_ii(A, B, N)), f"problem {q} {cases[q]} vs oracle"


@pytest.mark.parametrize("N,dtype", [(7, np.float64), (14, np.float64), (28, np.float64),
                                     (36, np.float64), (45, np.float64), (16, np.float32)])
def test_batched_one_residue_path(N, dtype):
    # Every problem takes the same residue path (one exact step, two limbs,
    # three limbs, three and four exact steps; FP32 on two limbs), so the
    # batch runs the grouped residue kernel built for that path alone.  A
    # problem of another N in the same batch brings back the per-tile choice.
    cases = [(70, 50, 90, N), (129, 257, 64, N), (33, 20, 300, N), (1, 3, 2, N)]
    announce(f"batched, one residue path: N={N} {np.dtype(dtype).name}")
    As, Bs = make_batch(cases, dtype, seed=300 + N)
    for Ns in ([N] * 4, [N, N, N, 2]):
        _, _, Ccm, _ = run_batched(As, Bs, Ns)
        assert oz.ozaki2_sync_status() == oz.OK
        for q, (A, B, Nq) in enumerate(zip(As, Bs, Ns)):
            got = host(Ccm[q]).T
            assert np.array_equal(got, single(A, B, Nq)), f"problem {q} {cases[q][:3]} N={Nq}"
            if q == 3:
                assert np.array_equal(got, os_ii(A, B, Nq)), f"problem {q} vs oracle"


@pytest.mark.parametrize("persist", [1, 0, 2])
@pytest.mark.parametrize("split", [0, 1000000, 4])
def test_batched_tile_splits_and_eager(split, persist):
    # Every tile split (all 256x256, all 128x128, mixed), the three forms of
    # the residue products (persistent workgroups walking the block map, one
    # workgroup per tile, one launch per problem) and the eager (uncaptured)
    # launch sequence give the same bits.
    announce(f"batched split={split} persist={persist}")
    cases = SMALL[:6] + SMALL[9:]
    As, Bs = make_batch(cases, np.float64, seed=300)
    Ns = [c[3] for c in cases]
    with oz.tuning(oz.KNOB_BATCH_SPLIT, split), oz.tuning(oz.KNOB_BATCH_PERSIST, persist):
        _, _, C1, _ = run_batched(As, Bs, Ns)
        with oz.tuning(oz.KNOB_BATCH_GRAPH, 0):
            _, _, C2, _ = run_batched(As, Bs, Ns)
    for q, (A, B, N) in enumerate(zip(As, Bs, Ns)):
        ref = single(A, B, N)
        assert np.array_equal(host(C1[q]).T, ref), f"graph, problem {q}"
        assert np.array_equal(host(C2[q]).T, ref), f"eager, problem {q}"


def test_batched_persistent_many_problems_and_long_k():
    # More entries than resident workgroups (each workgroup walks several
    # tiles of different problems and k), problems ordered by k, and one
    # problem with k > 2^17 (the build with reductions mod p inside k).
    cases = [(200 + 13 * q, 150 + 7 * q, 64 + 97 * q, 12 + q % 5) for q in range(40)]
    cases += [(24, 20, 2 ** 17 + 300, 14), (640, 512, 700, 16)]
    announce(f"batched persistent: {len(cases)} problems, one with k > 2^17")
    As, Bs = make_batch(cases, np.float64, seed=700)
    Ns = [c[3] for c in cases]
    with oz.tuning(oz.KNOB_BATCH_PERSIST, 1):
        _, _, Ccm, _ = run_batched(As, Bs, Ns)
    assert oz.ozaki2_sync_status() == oz.OK
    for q, (A, B, N) in enumerate(zip(As, Bs, Ns)):
        assert np.array_equal(host(Ccm[q]).T, single(A, B, N)), f"problem {q} {cases[q]}"
    q = len(cases) - 2
    rows, cols = np.array([0, 11, 23]), np.array([0, 19])
    assert np.array_equal(host(Ccm[q]).T[np.ix_(rows, cols)],
                          os_ii(As[q], Bs[q], Ns[q], rows=rows, cols=cols))


@pytest.mark.parametrize("persist,dtype", [(2, np.float64), (-1, np.float64), (2, np.float32)])
def test_batched_per_problem_split_k(persist, dtype):
    # Small outputs with long k: in the per-problem form each problem's
    # scaling and residue products split k (partials summed exactly, mod p for
    # the residues) as the single-problem call does.  Forced (2) and chosen by
    # the tuner (-1), the bits are those of the single calls and the oracle.
    cases = [(64, 48, 32768, 14), (30, 70, 20000, 12), (130, 5, 65536, 16), (1, 1, 40000, 7),
             (200, 180, 3000, 14), (17, 9, 2 ** 17 + 1000, 20)]
    if dtype == np.float32:
        cases = [(m, n, k, min(N, 16)) for m, n, k, N in cases]
    announce(f"batched per-problem split-k, persist={persist} {np.dtype(dtype).name}")
    As, Bs = make_batch(cases, dtype, seed=900)
    Ns = [c[3] for c in cases]
    with oz.tuning(oz.KNOB_BATCH_PERSIST, persist):
        A1, B1, C1, shapes = run_batched(As, Bs, Ns)
        first = [host(c).T for c in C1]
        with oz.tuning(oz.KNOB_BATCH_GRAPH, 0):
            _, _, C2, _ = run_batched(As, Bs, Ns)
        # the same buffers again: a replay of the captured graph, after other
        # work on the stream (the eager batch) and with C reset
        for c in C1:
            c.fill_(np.nan)
        oz.gemm_batched_cm(A1, B1, C1, shapes, Ns)
    assert oz.ozaki2_sync_status() == oz.OK
    for q, (A, B, N) in enumerate(zip(As, Bs, Ns)):
        ref = single(A, B, N)
        assert np.array_equal(first[q], ref), f"first call, problem {q} {cases[q]}"
        assert np.array_equal(host(C2[q]).T, ref), f"eager, problem {q} {cases[q]}"
        assert np.array_equal(host(C1[q]).T, ref), f"replay, problem {q} {cases[q]}"
    for q in (1, 3):
        assert np.array_equal(host(C1[q]).T, os_ii(As[q], Bs[q], Ns[q])), f"problem {q} vs oracle"
    rows, cols = np.array([0, 16]), np.array([0, 8])
    q = 5
    assert np.array_equal(host(C1[q]).T[np.ix_(rows, cols)],
                          os_ii(As[q], Bs[q], Ns[q], rows=rows, cols=cols))


def test_batched_graph_replays():
    # Same buffers three times: the first call captures, the next two replay.
    # Between replays: single-problem calls on the same stream (they reuse the
    # workspace), host synchronisation, and C reset to NaN.
    announce("batched graph replays")
    cases = [(300, 200, 500, 14), (129, 257, 64, 9), (512, 512, 256, 17)]
    As, Bs = make_batch(cases, np.float64, seed=500)
    Ns = [c[3] for c in cases]
    Acm, Bcm, Ccm, shapes = run_batched(As, Bs, Ns)
    refs = [single(A, B, N) for A, B, N in zip(As, Bs, Ns)]
    for rep in range(3):
        got = [host(C).T for C in Ccm]
        for q in range(len(cases)):
            assert np.array_equal(got[q], refs[q]), f"replay {rep} problem {q}"
        X, Y = gemm_inputs(200, 150, 300, seed=rep)
        _ = single(X, Y, 12)                        # eager work in between
        for C in Ccm:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        oz.gemm_batched_cm(Acm, Bcm, Ccm, shapes, Ns)
    assert oz.ozaki2_sync_status() == oz.OK


def test_batched_errors_and_nonfinite():
    announce("batched errors / non-finite")
    As, Bs = make_batch([(40, 30, 50, 10), (20, 20, 20, 12)], np.float64, seed=7)
    with pytest.raises(oz.Ozaki2Error) as ei:
        run_batched(As, Bs, [10, 50])              # N out of range in one problem
    assert ei.value.code == oz.ERR_N_RANGE
    A0 = As[0].copy()
    A0[3, 4] = np.inf
    _, _, Ccm, _ = run_batched([A0, As[1]], Bs, [10, 12])
    assert oz.ozaki2_sync_status() == oz.ERR_NONFINITE
    assert np.all(np.isnan(host(Ccm[0])))
    assert np.array_equal(host(Ccm[1]).T, single(As[1], Bs[1], 12))
    assert oz.ozaki2_sync_status() == oz.OK


def test_batched_512_workload_sampled():
    # The uneven 512-problem workload (m, n, k log-uniform in [64, 2048],
    # phi = 1, N per problem from the planner at 1e-15): every problem is
    # compared in full with the single-problem call, and four problems with
    # the oracle on sampled rows and columns.
    announce("batched 512-problem workload")
    shapes, mats = batched_inputs(512, phi=1.0, seed=0)
    dA = [cm(A) for A, _ in mats]
    dB = [cm(B) for _, B in mats]
    Ns = []
    for (m, n, k), a, b in zip(shapes, dA, dB):
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc, N = oz.ozaki2_required_moduli(64, m, n, k, a.data_ptr(), m, b.data_ptr(), k, 1e-15)
        assert rc in (oz.OK, oz.ERR_UNREACHABLE)
        Ns.append(N)
    print(f"[batched] N range {min(Ns)}..{max(Ns)}", flush=True)
    Ccm = [torch.full((n, m), float("nan"), dtype=torch.float64, device="cuda:0") for m, n, _ in shapes]
    oz.gemm_batched_cm(dA, dB, Ccm, shapes, Ns)
    assert oz.ozaki2_sync_status() == oz.OK
    rng = np.random.default_rng(1)
    for q in range(512):
        m, n, k = shapes[q]
        ref = torch.empty((n, m), dtype=torch.float64, device="cuda:0")
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        rc = oz.ozaki2_gemm(m, n, k, dA[q].data_ptr(), m, dB[q].data_ptr(), k, ref.data_ptr(), m, Ns[q])
        assert rc == oz.OK
        assert torch.equal(ref, Ccm[q]), f"problem {q} {shapes[q]} N={Ns[q]}"
    for q in rng.choice(512, 4, replace=False):
        m, n, k = shapes[q]
        rows = np.sort(rng.choice(m, min(m, 8), replace=False))
        cols = np.sort(rng.choice(n, min(n, 8), replace=False))
        want = os_ii(mats[q][0], mats[q][1], Ns[q], rows=rows, cols=cols)
        got = host(Ccm[q]).T[np.ix_(rows, cols)]
        assert np.array_equal(got, want), f"problem {q} vs oracle"


def test_caller_owned_workspace():
    # Single and batched calls on a caller-installed workspace of exactly the
    # queried size give the same bits as on the library's; one byte less is
    # refused before anything runs.
    announce("caller-owned workspace")
    A, B = gemm_inputs(300, 200, 500, seed=11)
    ref = single(A, B, 14)
    cases = [(300, 200, 500, 14), (64, 64, 64, 2), (5, 4, 0, 10)]
    As, Bs = make_batch(cases, np.float64, seed=12)
    Ns = [c[3] for c in cases]
    refs = [single(a, b, N) for a, b, N in zip(As, Bs, Ns)]   # on the library's workspace
    try:
        nbytes = oz.ozaki2_workspace_bytes(64, 300, 200, 500, 14)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        assert oz.ozaki2_set_workspace(ws.data_ptr(), nbytes) == oz.OK
        assert np.array_equal(single(A, B, 14), ref)
        assert oz.ozaki2_set_workspace(ws.data_ptr(), nbytes - 1) == oz.OK
        with pytest.raises(oz.Ozaki2Error) as ei:
            oz.gemm(dev(A), dev(B), 14)
        assert ei.value.code == oz.ERR_WORKSPACE
        need = oz.ozaki2_batched_workspace_bytes(64, [v for c in cases for v in c])
        wsb = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        assert oz.ozaki2_set_workspace(wsb.data_ptr(), need) == oz.OK
        _, _, Ccm, _ = run_batched(As, Bs, Ns)
        for q in range(len(cases)):
            assert np.array_equal(host(Ccm[q]).T, refs[q]), f"problem {q}"
        assert oz.ozaki2_set_workspace(wsb.data_ptr(), need - 1) == oz.OK
        with pytest.raises(oz.Ozaki2Error) as ei:
            run_batched(As, Bs, Ns)
        assert ei.value.code == oz.ERR_WORKSPACE
        torch.cuda.synchronize()
    finally:
        oz.ozaki2_set_workspace(None, 0)
