"""Python binding of libozaki2.so, the gfx950 Ozaki-II emulated GEMM.

Argument marshalling only: every step of the method runs in the HIP library.
The ``ozaki2_*`` functions mirror the C ABI of include/ozaki2.h (device
pointers as Python ints); ``gemm``/``sgemm``/``required_moduli``/
``debug_stages`` are torch conveniences that lay out column-major buffers
and pass torch's current stream to the library.

Importing this package does not touch the GPU; the library is loaded on first
use and a missing build raises immediately.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libozaki2.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_N_RANGE = -2
ERR_K_RANGE = -3
ERR_WORKSPACE = -4
ERR_UNREACHABLE = -5
ERR_NONFINITE = -6
ERR_HIP = -7
ERR_INIT = -8
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "N_RANGE", -3: "K_RANGE", -4: "WORKSPACE",
                -5: "UNREACHABLE", -6: "NONFINITE", -7: "HIP", -8: "INIT"}

_lib = None

_c_int, _c_size, _c_ptr, _c_double = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
_SIGS = {
    "ozaki2_gemm": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_sgemm": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_required_moduli": ([_c_int, _c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_double,
                                ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_debug_mfma_probe": ([_c_int, _c_int, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_c_double)],
                                _c_int),
    "ozaki2_zrequired_moduli": ([_c_int, _c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int,
                                 _c_double, ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_gemm_certified": ([_c_int, _c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int,
                               _c_double, _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(_c_double)], _c_int),
    "ozaki2_certified_workspace_bytes": ([_c_int, _c_int, _c_int, _c_int, _c_int], _c_size),
    "ozaki2_zgemm": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_cgemm": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_complex_workspace_bytes": ([_c_int, _c_int, _c_int, _c_int, _c_int], _c_size),
    "ozaki2_zgemm3m": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_cgemm3m": ([_c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int], _c_int),
    "ozaki2_set_stream": ([_c_ptr], _c_int),
    "ozaki2_set_moduli_table": ([_c_int], _c_int),
    "ozaki2_moduli": ([_c_int, _c_int, ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_debug_constants": ([_c_int, _c_int, _c_int, ctypes.POINTER(_c_double)], _c_int),
    "ozaki2_workspace_bytes": ([_c_int, _c_int, _c_int, _c_int, _c_int], _c_size),
    "ozaki2_set_workspace": ([_c_ptr, _c_size], _c_int),
    "ozaki2_sync_status": ([], _c_int),
    "ozaki2_gemm_noalloc": ([_c_int, _c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_ptr, _c_int,
                             _c_int], _c_int),
    "ozaki2_gemm_batched": ([_c_int, _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(_c_ptr),
                             ctypes.POINTER(_c_int), ctypes.POINTER(_c_ptr), ctypes.POINTER(_c_int),
                             ctypes.POINTER(_c_ptr), ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_batched_workspace_bytes": ([_c_int, _c_int, ctypes.POINTER(_c_int)], ctypes.c_size_t),
    "ozaki2_debug_stages": ([_c_int, _c_int, _c_int, _c_int, _c_ptr, _c_int, _c_ptr, _c_int, _c_int,
                             _c_int, ctypes.POINTER(_c_ptr)], _c_int),
    "ozaki2_debug_log2f": ([_c_ptr, _c_ptr, _c_int], _c_int),
    "ozaki2_profile": ([_c_int], _c_int),
    "ozaki2_profile_read": ([ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_float), _c_int], _c_int),
    "ozaki2_profile_name": ([_c_int], ctypes.c_char_p),
    "ozaki2_debug_tuning": ([_c_int, _c_int, ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_version": ([], ctypes.c_char_p),
}

KNOB_SLICE_WORKGROUPS, KNOB_GEMM_TILE, KNOB_BATCH_SPLIT, KNOB_BATCH_GRAPH, KNOB_BATCH_PERSIST = 0, 1, 2, 3, 4
KNOB_SPLIT_K = 5


class Ozaki2Error(RuntimeError):
    def __init__(self, func: str, code: int):
        super().__init__(f"{func} failed: {STATUS_NAMES.get(code, code)} ({code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libozaki2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _call(name, *args):
    return getattr(lib(), name)(*args)


# ---- C ABI mirrors (device pointers as ints) ------------------------------
def ozaki2_gemm(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_gemm", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_sgemm(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_sgemm", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_debug_mfma_probe(iters, changing=1):
    """(rc, ms, ops) of the MFMA-rate probe."""
    ms = ctypes.c_float(0.0)
    ops = _c_double(0.0)
    rc = _call("ozaki2_debug_mfma_probe", iters, changing, ctypes.byref(ms), ctypes.byref(ops))
    return rc, ms.value, ops.value


def ozaki2_zrequired_moduli(prec, m, n, k, A, lda, B, ldb, eps):
    out = _c_int(0)
    rc = _call("ozaki2_zrequired_moduli", prec, m, n, k, A, lda, B, ldb, eps, ctypes.byref(out))
    return rc, out.value


def ozaki2_required_moduli(prec, m, n, k, A, lda, B, ldb, eps):
    out = _c_int(0)
    rc = _call("ozaki2_required_moduli", prec, m, n, k, A, lda, B, ldb, eps, ctypes.byref(out))
    return rc, out.value


def ozaki2_gemm_certified(prec, m, n, k, A, lda, B, ldb, C, ldc, eps, N_start):
    """(rc, N_used, ratio)."""
    n_used, ratio = _c_int(0), _c_double(0.0)
    rc = _call("ozaki2_gemm_certified", prec, m, n, k, A, lda, B, ldb, C, ldc, eps, N_start,
               ctypes.byref(n_used), ctypes.byref(ratio))
    return rc, n_used.value, ratio.value


def ozaki2_certified_workspace_bytes(prec, m, n, k, N):
    return _call("ozaki2_certified_workspace_bytes", prec, m, n, k, N)


def ozaki2_zgemm(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_zgemm", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_cgemm(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_cgemm", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_zgemm3m(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_zgemm3m", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_cgemm3m(m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_cgemm3m", m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_complex_workspace_bytes(prec, m, n, k, N):
    return _call("ozaki2_complex_workspace_bytes", prec, m, n, k, N)


def ozaki2_set_stream(stream):
    return _call("ozaki2_set_stream", stream)


MODULI_PAPER, MODULI_OPTIMAL = 0, 1


def ozaki2_set_moduli_table(table):
    return _call("ozaki2_set_moduli_table", table)


def ozaki2_moduli(table, N):
    """(rc, list of the N moduli)."""
    out = (_c_int * max(N, 1))()
    rc = _call("ozaki2_moduli", table, N, out)
    return rc, list(out)[:N] if rc == OK else []


def ozaki2_debug_constants(prec, table, N):
    """(rc, dict with P1, P2, Pinv, Pprime, c, s1, s2)."""
    out = (_c_double * (5 + 2 * max(N, 0)))()
    rc = _call("ozaki2_debug_constants", prec, table, N, out)
    if rc != OK:
        return rc, None
    v = list(out)
    return rc, {"P1": v[0], "P2": v[1], "Pinv": v[2], "Pprime": v[3], "c": v[4],
                "s1": v[5:5 + N], "s2": v[5 + N:5 + 2 * N]}


class moduli_table:
    """Context manager: calls on this thread use `table` inside the block."""

    def __init__(self, table):
        self.table = table

    def __enter__(self):
        rc = ozaki2_set_moduli_table(self.table)
        if rc != OK:
            raise Ozaki2Error("ozaki2_set_moduli_table", rc)
        return self

    def __exit__(self, *exc):
        ozaki2_set_moduli_table(MODULI_PAPER)
        return False


def ozaki2_workspace_bytes(prec, m, n, k, N):
    return _call("ozaki2_workspace_bytes", prec, m, n, k, N)


def ozaki2_set_workspace(ptr, nbytes):
    return _call("ozaki2_set_workspace", ptr, nbytes)


def ozaki2_sync_status():
    return _call("ozaki2_sync_status")


def ozaki2_gemm_noalloc(prec, m, n, k, A, lda, B, ldb, C, ldc, N):
    return _call("ozaki2_gemm_noalloc", prec, m, n, k, A, lda, B, ldb, C, ldc, N)


def ozaki2_gemm_batched(prec, mnkN, A, lda, B, ldb, C, ldc):
    count = len(A)
    arr_i = lambda v: (_c_int * len(v))(*v)
    arr_p = lambda v: (_c_ptr * len(v))(*v)
    return _call("ozaki2_gemm_batched", prec, count, arr_i(mnkN), arr_p(A), arr_i(lda), arr_p(B),
                 arr_i(ldb), arr_p(C), arr_i(ldc))


def ozaki2_batched_workspace_bytes(prec, mnkN):
    count = len(mnkN) // 4
    return lib().ozaki2_batched_workspace_bytes(prec, count, (_c_int * max(len(mnkN), 1))(*mnkN))


def ozaki2_debug_stages(prec, m, n, k, A, lda, B, ldb, N, outs):
    arr = (_c_ptr * len(outs))(*[o or None for o in outs])
    return _call("ozaki2_debug_stages", prec, m, n, k, A, lda, B, ldb, N, len(outs), arr)


def ozaki2_debug_log2f(d, out, count):
    return _call("ozaki2_debug_log2f", d, out, count)


def ozaki2_profile(enable):
    return _call("ozaki2_profile", enable)


def ozaki2_profile_read(cap=4096):
    ph = (_c_int * cap)()
    ms = (ctypes.c_float * cap)()
    n = _call("ozaki2_profile_read", ph, ms, cap)
    if n < 0:
        raise Ozaki2Error("ozaki2_profile_read", n)
    names = [lib().ozaki2_profile_name(ph[i]).decode() for i in range(n)]
    return list(zip(names, [ms[i] for i in range(n)]))


def ozaki2_debug_tuning(knob, value):
    """(rc, previous value)."""
    prev = _c_int(0)
    rc = _call("ozaki2_debug_tuning", knob, value, ctypes.byref(prev))
    return rc, prev.value


class tuning:
    """Context manager: set a knob of ozaki2_debug_tuning, restore it on exit."""

    def __init__(self, knob, value):
        self.knob, self.value, self.prev = knob, value, None

    def __enter__(self):
        rc, self.prev = ozaki2_debug_tuning(self.knob, self.value)
        if rc != OK:
            raise Ozaki2Error("ozaki2_debug_tuning", rc)
        return self

    def __exit__(self, *exc):
        ozaki2_debug_tuning(self.knob, self.prev)
        return False


def ozaki2_version():
    return lib().ozaki2_version().decode()


# ---- torch conveniences (layout + stream only) -----------------------------
def _torch():
    import torch
    return torch


def _set_current_stream():
    torch = _torch()
    ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)


def col_major(X):
    """Column-major device copy of a logical (r x c) matrix: a (c x r)
    contiguous tensor whose data is X in column-major order (ld = r)."""
    return X.t().contiguous()


def gemm(A, B, N: int, out=None):
    """C = A @ B (logical shapes) by the FP64 or FP32 emulation with N moduli.
    A, B: CUDA tensors of equal dtype (float64 / float32).  Returns C (m x n),
    a transposed view of a column-major buffer."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    Acm, Bcm = col_major(A), col_major(B)
    Ccm = out if out is not None else torch.empty((n, m), dtype=A.dtype, device=A.device)
    _set_current_stream()
    f = ozaki2_gemm if A.dtype == torch.float64 else ozaki2_sgemm
    rc = f(m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(), max(k, 1), Ccm.data_ptr(), max(m, 1), N)
    if rc != OK:
        raise Ozaki2Error("ozaki2_gemm", rc)
    return Ccm.t()


def zgemm(A, B, N: int, form: str = "4m"):
    """C = A @ B for complex CUDA tensors (complex128: ozaki2_zgemm,
    complex64: ozaki2_cgemm; form="3m": ozaki2_zgemm3m / ozaki2_cgemm3m).
    Returns C (m x n), a transposed view of a column-major buffer."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    Acm, Bcm = col_major(A), col_major(B)
    Ccm = torch.empty((n, m), dtype=A.dtype, device=A.device)
    _set_current_stream()
    if form == "3m":
        f = ozaki2_zgemm3m if A.dtype == torch.complex128 else ozaki2_cgemm3m
    elif form == "4m":
        f = ozaki2_zgemm if A.dtype == torch.complex128 else ozaki2_cgemm
    else:
        raise ValueError(f"form must be '4m' or '3m', not {form!r}")
    rc = f(m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(), max(k, 1), Ccm.data_ptr(), max(m, 1), N)
    if rc != OK:
        raise Ozaki2Error("ozaki2_zgemm", rc)
    return Ccm.t()


def required_moduli(A, B, eps: float):
    """(rc, N) from ozaki2_required_moduli for logical A (m x k), B (k x n);
    complex tensors go to ozaki2_zrequired_moduli (the real embedding)."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    Acm, Bcm = col_major(A), col_major(B)
    _set_current_stream()
    if A.dtype in (torch.complex128, torch.complex64):
        prec = 64 if A.dtype == torch.complex128 else 32
        return ozaki2_zrequired_moduli(prec, m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(),
                                       max(k, 1), eps)
    prec = 64 if A.dtype == torch.float64 else 32
    return ozaki2_required_moduli(prec, m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(), max(k, 1), eps)


def gemm_certified(A, B, eps: float, N_start: int = 0):
    """(C, rc, N_used, ratio) from ozaki2_gemm_certified for logical A (m x k), B (k x n);
    C is A @ B at N_used as a (transposed view of a) column-major tensor."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    Acm, Bcm = col_major(A), col_major(B)
    Ccm = torch.empty((n, m), dtype=A.dtype, device=A.device)
    _set_current_stream()
    prec = 64 if A.dtype == torch.float64 else 32
    rc, N, ratio = ozaki2_gemm_certified(prec, m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(),
                                         max(k, 1), Ccm.data_ptr(), max(m, 1), eps, N_start)
    return Ccm.t(), rc, N, ratio


def debug_stages(A, B, N: int, crt_stages: bool = True):
    """Every intermediate of Algorithms 1-3 as torch tensors (see the header);
    with crt_stages, also the INT32 products C'_l and C'(1), C'(2), Q, C''."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    dev = A.device
    i32 = dict(dtype=torch.int32, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    out = dict(mu_p=torch.empty(m, **i32), nu_p=torch.empty(n, **i32), rmax=torch.empty(m, **i32),
               cmax=torch.empty(n, **i32), mu=torch.empty(m, **i32), nu=torch.empty(n, **i32),
               Al=torch.empty((N, m, k), dtype=torch.int8, device=dev),
               BlT=torch.empty((N, n, k), dtype=torch.int8, device=dev),
               WT=torch.empty((N, n, m), dtype=torch.int8, device=dev),
               CT=torch.empty((n, m), dtype=A.dtype, device=dev),
               ef=torch.empty(m + n, dtype=torch.float32, device=dev))
    order = ["mu_p", "nu_p", "rmax", "cmax", "mu", "nu", "Al", "BlT", "WT", "CT", "ef"]
    if crt_stages:
        out.update(ClT=torch.empty((N, n, m), **i32), C1T=torch.empty((n, m), **f64),
                   C2T=torch.empty((n, m), **f64), QT=torch.empty((n, m), **f64),
                   CppT=torch.empty((n, m), **f64))
        order += ["ClT", "C1T", "C2T", "QT", "CppT"]
    Acm, Bcm = col_major(A), col_major(B)
    _set_current_stream()
    prec = 64 if A.dtype == torch.float64 else 32
    rc = ozaki2_debug_stages(prec, m, n, k, Acm.data_ptr(), max(m, 1), Bcm.data_ptr(), max(k, 1), N,
                             [out[o].data_ptr() for o in order])
    if rc != OK:
        raise Ozaki2Error("ozaki2_debug_stages", rc)
    return out


def gemm_batched_cm(Acm, Bcm, Ccm, shapes, Ns):
    """One ozaki2_gemm_batched call on column-major device buffers.

    Acm[p], Bcm[p], Ccm[p]: tensors holding A_p (m x k), B_p (k x n), C_p (m x n)
    in column-major order (as made by col_major); shapes[p] = (m, n, k);
    Ns[p] = moduli count.  The same buffers on a later call replay the
    captured launch sequence."""
    torch = _torch()
    if not Acm:
        return
    prec = 64 if Acm[0].dtype == torch.float64 else 32
    mnkN, la, lb, lc = [], [], [], []
    for (m, n, k), N in zip(shapes, Ns):
        mnkN += [m, n, k, N]
        la.append(max(m, 1))
        lb.append(max(k, 1))
        lc.append(max(m, 1))
    _set_current_stream()
    rc = ozaki2_gemm_batched(prec, mnkN, [a.data_ptr() for a in Acm], la,
                             [b.data_ptr() for b in Bcm], lb, [c.data_ptr() for c in Ccm], lc)
    if rc != OK:
        raise Ozaki2Error("ozaki2_gemm_batched", rc)


def gemm_batched(As, Bs, Ns):
    """[A_p @ B_p] for logical A_p (m x k), B_p (k x n) by one batched call."""
    torch = _torch()
    shapes = [(A.shape[0], B.shape[1], A.shape[1]) for A, B in zip(As, Bs)]
    Acm = [col_major(A) for A in As]
    Bcm = [col_major(B) for B in Bs]
    Ccm = [torch.empty((n, m), dtype=A.dtype, device=A.device) for (m, n, _), A in zip(shapes, As)]
    gemm_batched_cm(Acm, Bcm, Ccm, shapes, Ns)
    return [C.t() for C in Ccm]
