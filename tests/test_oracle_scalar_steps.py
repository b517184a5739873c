"""Pins of Algorithm 2's scalar steps in the oracle: Dbar = single_up(Cbar)
(the row / column maxima rounded up to FP32) and e = log2f(Dbar) in its
vectorised form, each against a computation that does not use the oracle's
own rounding code, plus planted mistakes that these pins must catch."""
import numpy as np

import oracle.ozaki2 as oz
from oracle.fp import round_f32
from pins import (log2f_near_midpoint_inputs, pin_log2f_many, pin_single_up, single_up_cases,
                  single_up_reference)


def test_single_up_reference_is_sound():
    # The reference itself: exact below 2^24, a multiple of the FP32 spacing
    # above, never below M and less than one spacing above it.
    M = single_up_cases(seed=3)
    ref = single_up_reference(M)
    assert np.all(ref >= M)
    small = M <= 2 ** 24
    assert np.array_equal(ref[small], M[small])
    big = ~small
    spacing = 2 ** (np.floor(np.log2(ref[big].astype(np.float64))).astype(np.int64) - 23)
    assert np.all(ref[big] % spacing == 0)
    assert np.all(ref[big] - M[big] < np.maximum(spacing, 1))


def test_single_up_int_pinned():
    # Algorithm 2: Dbar = single_up(Cbar), on every M in (2^24, 2^24 + 2^12],
    # the grid neighbours of FP32 values up to 2^32 and random M up to 2^32.
    assert pin_single_up(oz.single_up_int, single_up_cases(seed=0)) == []


def test_single_up_round_down_is_caught():
    wrong = lambda M: int(round_f32(M, "rd")) if M > 0 else 0
    assert pin_single_up(wrong, single_up_cases(seed=1)) != []


def test_single_up_round_nearest_is_caught():
    wrong = lambda M: int(round_f32(M, "rn")) if M > 0 else 0
    assert pin_single_up(wrong, single_up_cases(seed=2)) != []


def _log2f_inputs():
    rng = np.random.default_rng(17)
    near = log2f_near_midpoint_inputs(1, 2 ** 24)          # every near-midpoint input up to 2^24
    rand = rng.integers(1, 2 ** 24, 6000).astype(np.float64)
    wide = (rng.integers(2 ** 23, 2 ** 24, 4000) << rng.integers(1, 9, 4000)).astype(np.float64)
    pw = np.array([2.0 ** e for e in range(33)])
    d = np.concatenate([near, rand, wide, pw, pw[1:] - 1, pw[:25] + 1])
    return d, near


def test_log2f_many_matches_scalar_log2f():
    # R6: the vectorised form used by the exhaustive GPU check equals the
    # decimal-pinned scalar log2f on >= 10^4 inputs, among them every input
    # up to 2^24 that it settles through its near-midpoint path.
    d, near = _log2f_inputs()
    assert near.size > 50
    assert d.size >= 10 ** 4
    assert pin_log2f_many(oz.log2f_many, d) == []


def test_log2f_many_truncation_is_caught():
    def wrong(d):
        v = np.log2(np.asarray(d, dtype=np.float64))
        r = v.astype(np.float32)
        over = r.astype(np.float64) > v                     # round toward zero instead of nearest
        r[over] = np.nextafter(r[over], np.float32(0))
        return r
    d, _ = _log2f_inputs()
    assert pin_log2f_many(wrong, d[:3000]) != []


def test_log2f_many_wrong_midpoint_choice_is_caught():
    # A near-midpoint path that picks the other neighbour must be seen on the
    # near-midpoint inputs.
    def wrong(d):
        d = np.asarray(d, dtype=np.float32)
        out = oz.log2f_many(d)
        v = np.log2(d.astype(np.float64))
        r = v.astype(np.float32)
        rd = r.astype(np.float64)
        up = np.nextafter(r, np.float32(np.inf)).astype(np.float64)
        dn = np.nextafter(r, np.float32(-np.inf)).astype(np.float64)
        tol = np.abs(v) * 2.0 ** -40
        nu = np.abs(v - 0.5 * (rd + up)) <= tol
        nd = np.abs(v - 0.5 * (rd + dn)) <= tol
        out[nu] = np.where(out[nu] == r[nu], np.nextafter(r[nu], np.float32(np.inf)), r[nu])
        out[nd] = np.where(out[nd] == r[nd], np.nextafter(r[nd], np.float32(-np.inf)), r[nd])
        return out
    _, near = _log2f_inputs()
    assert pin_log2f_many(wrong, near) != []
