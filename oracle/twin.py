"""Loader of the C++ twin of the oracle (oracle/os_ii_twin.cpp).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The twin implements
Algorithms 1-3 with plain loops and OpenMP; the constants of Section 3.1 are
passed in from oracle/constants.py.  It serves as a second implementation
that the Python oracle is compared with stage by stage, and as the CPU
timing of the oracle on every host core.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .constants import constants

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "os_ii_twin.cpp")
LIB = os.path.join(HERE, "libos_ii_twin.so")

_lib = None


def build() -> str:
    """Compile the twin with g++ (OpenMP; no contraction of a*b+c into fma,
    so every fused multiply-add is an explicit one)."""
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", SRC,
           "-o", tmp]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.ozaki2_oracle_twin.argtypes = ([ctypes.c_int] * 4 + [P, P, ctypes.c_int, P, P, P]
                                         + [ctypes.c_double] * 5 + [P] * 14)
        L.ozaki2_oracle_twin.restype = ctypes.c_int
        L.ozaki2_oracle_twin_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the twin's loops run on."""
    return int(lib().ozaki2_oracle_twin_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def os_ii_twin(A: np.ndarray, B: np.ndarray, N: int, stages: bool = False, table: str = "paper"):
    """C := OS_II(A, B, p) by the C++ twin (same conventions as
    oracle.ozaki2.os_ii; with stages=True also every intermediate)."""
    if A.dtype != B.dtype or A.dtype not in (np.float64, np.float32):
        raise ValueError("A and B must both be float64 or both float32")
    b = 64 if A.dtype == np.float64 else 32
    const = constants(N, b, table)
    m, k = A.shape
    n = B.shape[1]
    Ad = np.ascontiguousarray(A, dtype=np.float64)
    Bd = np.ascontiguousarray(B, dtype=np.float64)
    p = np.array(const.p, dtype=np.int32)
    s1 = np.array(const.s1, dtype=np.float64)
    s2 = np.array(const.s2, dtype=np.float64)
    C = np.empty((m, n), dtype=np.float64)
    st = None
    if stages:
        st = dict(mu_p=np.empty(m, np.int32), nu_p=np.empty(n, np.int32),
                  rmax=np.empty(m, np.int64), cmax=np.empty(n, np.int64),
                  mu=np.empty(m, np.int32), nu=np.empty(n, np.int32),
                  Al=np.empty((N, m, k), np.int8), Bl=np.empty((N, k, n), np.int8),
                  W=np.empty((N, m, n), np.int8), C1=np.empty((m, n)), C2=np.empty((m, n)),
                  Q=np.empty((m, n)), Cpp=np.empty((m, n)))
    g = (lambda key: _ptr(st[key])) if stages else (lambda key: None)
    rc = lib().ozaki2_oracle_twin(
        b, m, n, k, _ptr(Ad), _ptr(Bd), N, _ptr(p), _ptr(s1), _ptr(s2), const.P1, const.P2,
        const.Pinv, float(const.Pprime), float(const.c), g("mu_p"), g("nu_p"), g("rmax"),
        g("cmax"), g("mu"), g("nu"), g("Al"), g("Bl"), g("W"), g("C1"), g("C2"), g("Q"),
        g("Cpp"), _ptr(C))
    if rc != 0:
        raise ValueError(f"oracle twin failed with code {rc}")
    out = C if b == 64 else C.astype(np.float32)
    return (out, st) if stages else out
