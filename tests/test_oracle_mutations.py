"""Planted mistakes in the oracle (on the CPU): each plausible error in a step
of Algorithms 1-3 must make at least one pin fail.  This shows the pins are
sensitive enough to trust the oracle they accept."""
import dataclasses

import numpy as np
import pytest

import oracle.ozaki2 as oz
from pins import all_pins, fold_inputs, pin_residues
from workload import gemm_inputs, wrap_inputs


def _const_mut(monkeypatch, fn):
    real = oz.constants

    def patched(N, b=64, table="paper"):
        return fn(real(N, b, table))
    monkeypatch.setattr(oz, "constants", patched)


def m_s2_sign(mp):
    _const_mut(mp, lambda c: dataclasses.replace(c, s2=tuple(-v for v in c.s2)))


def m_drop_P2(mp):
    _const_mut(mp, lambda c: dataclasses.replace(c, P2=0.0))


def m_wrong_q(mp):
    def f(c):
        q = tuple((v % (p - 1)) + 1 if p > 2 else v for v, p in zip(c.q, c.p))
        q = (q[0],) + (q[1] % (c.p[1] - 1) + 1,) + q[2:]
        x = tuple((c.P // p) * v for p, v in zip(c.p, q))
        return dataclasses.replace(c, q=q, x=x)
    _const_mut(mp, f)


def m_shift_plus_one(mp):
    real = oz.shift
    mp.setattr(oz, "shift", lambda a, b, c: real(a, b, c) + 1)


def m_floor_mod(mp):
    mp.setattr(oz, "mod_sym", lambda X, p: np.asarray(np.mod(X, p)).astype(np.int64))


def m_transposed_operand(mp):
    real = oz.exact_int_matmul

    def f(X, Y, bound):
        if bound == 128.0 * 128.0 * max(X.shape[1], 1):
            return real(X, Y.T.copy(), bound)
        return real(X, Y, bound)
    mp.setattr(oz, "exact_int_matmul", f)


def m_floor_instead_of_ceil(mp):
    def f(absX, shift):
        v = np.floor(np.ldexp(absX, shift.astype(np.int32)))
        return v.astype(np.int64)
    mp.setattr(oz, "ceil_scaled", f)


def m_unscale_sign(mp):
    real = oz.unscale
    mp.setattr(oz, "unscale", lambda C, mu, nu, b: real(C, -mu + 2 * mu.min(), nu, b))


def m_drop_C2(mp):
    real = oz.crt_reconstruct

    def f(W, const):
        out = real(W, const)
        if const.b == 64:
            out = dict(out)
            out["C2"] = np.zeros_like(out["C2"])
        return out
    mp.setattr(oz, "crt_reconstruct", f)


def m_saturate_int32(mp):
    mp.setattr(oz, "wrap_int32", lambda X: np.clip(X, -2 ** 31, 2 ** 31 - 1))


MUTATIONS = [m_s2_sign, m_drop_P2, m_wrong_q, m_shift_plus_one, m_floor_mod,
             m_transposed_operand, m_floor_instead_of_ceil, m_unscale_sign]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda f: f.__name__)
def test_planted_mistake_is_caught(monkeypatch, mutation):
    mutation(monkeypatch)
    A, B = gemm_inputs(6, 6, 6, phi=1.0, seed=21)
    try:
        _, st = oz.os_ii(A, B, 14, stages=True)
    except AssertionError:
        return          # the oracle's own run-time assertions caught it
    assert all_pins(A, B, st) != []


def test_dropping_C2_is_caught(monkeypatch):
    # C'(2) carries only the low part of the CRT sum; dropping it must break
    # Lemma 2 (and Lemma 4) at N = 14.
    m_drop_C2(monkeypatch)
    A, B = gemm_inputs(6, 6, 6, phi=1.0, seed=22)
    _, st = oz.os_ii(A, B, 14, stages=True)
    assert all_pins(A, B, st) != []


def test_saturating_accumulator_is_caught(monkeypatch):
    # An INT32 accumulator that saturates instead of wrapping gives 2^31 - 1
    # for the p = 256 product at k = 2^17, which is not congruent to A'B'
    # modulo 256; the residue pin must see it.
    m_saturate_int32(monkeypatch)
    A, B = wrap_inputs(4, 3, 2 ** 17, seed=1)
    _, st = oz.os_ii(A, B, 14, stages=True)
    assert pin_residues(st) != []


def test_unchunked_int32_accumulation_is_caught(monkeypatch):
    # Reading R22: beyond 2^17 of k each residue product is formed in chunks
    # that stay exact in INT32.  A version that accumulates all of k in one
    # INT32 value wraps on the fold-stressing inputs (k = 2^18, all residues
    # mod 255 equal to +-127); the residue pin must see it.
    real = oz.residue_products

    def unchunked(Ap, Bp, const):
        out = real(Ap, Bp, const)
        W = []
        for l, p in enumerate(const.p):
            c = oz.wrap_int32(oz.exact_int_matmul(out["Al"][l], out["Bl"][l], 128.0 * 128.0 * Ap.shape[1]))
            W.append(oz.mod_sym(c, p))
        return dict(out, W=W)
    monkeypatch.setattr(oz, "residue_products", unchunked)
    A, B = fold_inputs(2, 3, 2 ** 18, 14)
    _, st = oz.os_ii(A, B, 14, stages=True)
    assert pin_residues(st) != []
