"""Per-N moduli that maximise P (Section 3.1, "Determination of Constants").

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.1 fixes one list of 49 pairwise coprime moduli p_l <= 256 and uses
its first N entries, but notes that the set maximising P = prod p_l depends
on N (255 drops out beyond a small N) and that a table per N can be built.
This module finds, for each N, N pairwise coprime integers in [2, 256] with
the largest product, by an exact branch-and-bound search:

  * Candidates: an integer v is dropped when some w in (v, 256] has every
    prime factor among v's.  Replacing v by such a w keeps the set pairwise
    coprime and raises P, so an optimal set never needs v.
  * Depth-first over candidates in descending order (take / skip), with the
    exact integer bound: the current product times the product of the r
    largest remaining candidates coprime to every prime used so far, r the
    number still to pick.  A branch is cut only when that bound is below the
    best product found (ties are explored), so the search is exhaustive.
  * Ties between sets of equal P (equal prime-power content grouped
    differently) are broken towards the lexicographically larger sequence in
    descending order, so the result is unique.

The set is returned in descending order (the order of the paper's list); the
order fixes the C'(2) accumulation order of Algorithm 3 (reading R11).
"""
from __future__ import annotations

from functools import lru_cache

P_MAX = 256


def prime_factors(v: int) -> frozenset:
    out, d = set(), 2
    while d * d <= v:
        while v % d == 0:
            out.add(d)
            v //= d
        d += 1
    if v > 1:
        out.add(v)
    return frozenset(out)


@lru_cache(maxsize=None)
def candidates() -> tuple:
    """Undominated integers in [2, 256], descending, with their prime sets."""
    supp = {v: prime_factors(v) for v in range(2, P_MAX + 1)}
    keep = []
    for v in range(P_MAX, 1, -1):
        if any(supp[w] <= supp[v] for w in range(v + 1, P_MAX + 1)):
            continue
        keep.append((v, supp[v]))
    return tuple(keep)


@lru_cache(maxsize=None)
def optimal_moduli(N: int) -> tuple:
    """N pairwise coprime integers in [2, 256] of largest product (descending)."""
    if not (1 <= N <= 49):
        raise ValueError("N must be in [1, 49]")
    cand = candidates()
    C = len(cand)
    best = [0, ()]                     # product, descending tuple

    def bound(start: int, used: frozenset, r: int) -> int:
        if r == 0:
            return 1
        prod, got = 1, 0
        for t in range(start, C):
            v, s = cand[t]
            if not (s & used):
                prod *= v
                got += 1
                if got == r:
                    return prod
        return 0                       # fewer than r usable candidates remain

    def dfs(start: int, used: frozenset, cur: int, chosen: tuple) -> None:
        r = N - len(chosen)
        if r == 0:
            if cur > best[0] or (cur == best[0] and chosen > best[1]):
                best[0], best[1] = cur, chosen
            return
        for t in range(start, C):
            # the bound only falls as t advances: nothing later can do better
            if cur * bound(t, used, r) < best[0]:
                break
            v, s = cand[t]
            if s & used:
                continue
            if cur * v * bound(t + 1, used | s, r - 1) < best[0]:
                continue
            dfs(t + 1, used | s, cur * v, chosen + (v,))

    dfs(0, frozenset(), 1, ())
    if len(best[1]) != N:
        raise ValueError(f"no {N} pairwise coprime moduli <= 256")
    return best[1]
