"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws matrices.

Recipe (the paper's experimental setup, Section 5): every entry is
(rand - 0.5) * exp(phi * randn), rand uniform, randn standard normal;
phi controls the exponent spread.  numpy's PCG64 generator
(``default_rng(seed)``) draws, per matrix, first the uniform array then the
normal array, in row-major order of the matrix's logical shape; A is drawn
before B.  FP32 inputs are the FP64 draws rounded to nearest.
"""
from __future__ import annotations

import math

import numpy as np


def draw_matrix(rng: np.random.Generator, shape, phi: float) -> np.ndarray:
    U = rng.random(shape)
    Z = rng.standard_normal(shape)
    return (U - 0.5) * np.exp(phi * Z)


def gemm_inputs(m: int, n: int, k: int, phi: float = 0.5, seed: int = 0,
                dtype=np.float64):
    """A (m x k) and B (k x n) for one emulated GEMM."""
    rng = np.random.default_rng(seed)
    A = draw_matrix(rng, (m, k), phi)
    B = draw_matrix(rng, (k, n), phi)
    return A.astype(dtype), B.astype(dtype)


def complex_gemm_inputs(m: int, n: int, k: int, phi: float = 0.5, seed: int = 0,
                        dtype=np.complex128):
    """Complex A (m x k) and B (k x n): the real recipe applied to each part.
    Draw order: A's real part, A's imaginary part, B's real part, B's
    imaginary part (each uniform array, then normal array).  complex64
    inputs are the complex128 draws with each part rounded to nearest."""
    rng = np.random.default_rng(seed)
    Ar, Ai = draw_matrix(rng, (m, k), phi), draw_matrix(rng, (m, k), phi)
    Br, Bi = draw_matrix(rng, (k, n), phi), draw_matrix(rng, (k, n), phi)
    return (Ar + 1j * Ai).astype(dtype), (Br + 1j * Bi).astype(dtype)


def batched_shapes(count: int = 512, lo: int = 64, hi: int = 2048, seed: int = 0):
    """(m, n, k) per problem, each log-uniform in [lo, hi], drawn in the order
    m, n, k per problem before any matrix.  Returns (rng, shapes) so that the
    caller can continue drawing the matrices from the same stream."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        mnk = [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(3)]
        shapes.append(tuple(mnk))
    return rng, shapes


def batched_inputs(count: int = 512, phi: float = 1.0, seed: int = 0, dtype=np.float64):
    """Uneven batch: list of (A, B) pairs, shapes from batched_shapes."""
    rng, shapes = batched_shapes(count, seed=seed)
    out = []
    for (m, n, k) in shapes:
        A = draw_matrix(rng, (m, k), phi).astype(dtype)
        B = draw_matrix(rng, (k, n), phi).astype(dtype)
        out.append((A, B))
    return shapes, out


def wrap_inputs(m: int, n: int, k: int, seed: int = 0, spread: int = 20):
    """Structured A (m x k) and B (k x n) whose entries are
    +-(1 + 2^-39) * 2^e, with a random sign per entry and one random integer
    exponent e in [-spread, spread] per row of A and per column of B.

    Every row of A and column of B then has the same significand pattern, so
    the scaled integers A', B' share one residue pattern modulo a power of
    two; at suitable N and k this drives INT32 accumulation of a residue
    product to its limit (used for the k = 2^17 wrap-around case)."""
    rng = np.random.default_rng(seed)
    u = 1.0 + 2.0 ** -39
    A = u * rng.choice([-1.0, 1.0], (m, k)) * np.ldexp(1.0, rng.integers(-spread, spread + 1, (m, 1)))
    B = u * rng.choice([-1.0, 1.0], (k, n)) * np.ldexp(1.0, rng.integers(-spread, spread + 1, (1, n)))
    return A, B
