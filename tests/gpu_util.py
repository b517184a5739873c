"""Helpers for the GPU parity tests (marshalling and oracle comparisons)."""
from __future__ import annotations

import sys

import numpy as np

from oracle.ozaki2 import log2f, single_up_int


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def oracle_e(cmax) -> np.ndarray:
    """e / f of Algorithm 2 from the oracle's row / column maxima of Cbar."""
    return np.array([float(log2f(single_up_int(max(int(M), 1)))) for M in cmax], dtype=np.float32)


def compare_stages(got: dict, st: dict, C_ref: np.ndarray, N: int) -> list:
    """Element-by-element comparison of every stage; returns failure strings."""
    bad = []

    def eq(name, a, b):
        a, b = np.asarray(a), np.asarray(b)
        if a.shape != b.shape:
            bad.append(f"{name}: shape {a.shape} vs {b.shape}")
        elif not np.array_equal(a, b):
            nd = int(np.sum(a != b))
            bad.append(f"{name}: {nd} of {a.size} differ")

    eq("mu'", got["mu_p"], st["mu_p"])
    eq("nu'", got["nu_p"], st["nu_p"])
    eq("row max Cbar", got["rmax"], st["rmax"])
    eq("col max Cbar", got["cmax"], st["cmax"])
    eq("mu", got["mu"], st["mu"])
    eq("nu", got["nu"], st["nu"])
    m = len(st["mu"])
    eq("e (log2f)", got["ef"][:m], oracle_e(st["rmax"]))
    eq("f (log2f)", got["ef"][m:], oracle_e(st["cmax"]))
    for l in range(N):
        eq(f"A'_{l}", got["Al"][l], st["Al"][l])
        eq(f"B'_{l}", got["BlT"][l], st["Bl"][l].T)
        eq(f"W_{l}", got["WT"][l], st["W"][l].T)
        if "ClT" in got:      # the INT32 residue products, two's complement
            if st["Al"][l].shape[1] <= 2 ** 17:
                eq(f"C'_{l}", got["ClT"][l].astype(np.int64), st["Cl"][l].T)
            else:             # reduced mod p_l every 2^17 of k: congruent only
                p = int(st["const"].p[l])
                eq(f"C'_{l} mod {p}", np.mod(got["ClT"][l].astype(np.int64), p),
                   np.mod(st["Cl"][l].T, p))
    if "C1T" in got:          # Algorithm 3's FP64 intermediates (Lemmas 2-4)
        eq("C'(1)", got["C1T"].T, st["C1"])
        eq("C'(2)", got["C2T"].T, st["C2"])
        eq("Q", got["QT"].T, st["Q"])
        eq("C''", got["CppT"].T, st["Cpp"])
    eq("C", got["CT"].T, C_ref)
    return bad


def rel_close(got: np.ndarray, ref: np.ndarray, rel: float) -> np.ndarray:
    """Entrywise |got - ref| <= rel * |ref| (exact zeros must match)."""
    g = got.astype(np.float64)
    r = ref.astype(np.float64)
    return np.abs(g - r) <= rel * np.abs(r)
