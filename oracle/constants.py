"""Constants of the Ozaki-II scheme, Section 3.1 "Determination of Constants".

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Everything here is computed from its definition with exact big integers;
the only transcendental quantity, P' (Algorithm 2, first step), is evaluated
with mpmath at 256-bit precision and then rounded down to FP32, with a check
that the working precision cannot change the rounding.

Readings (where the paper is silent or garbled):
  * the N moduli are the first N entries of the fixed 49-entry list of
    Section 3.1 (eq. p_list), or, with table="optimal", the per-N set of
    largest product that Section 3.1 says can be tabulated (oracle/moduli.py);
  * s_l1 keeps the upper beta_l bits of (P/p_l)*q_l by TRUNCATION, i.e. it is
    floor(x_l / g) * g with g = 2^(floor(log2 r) + 1 + ceil(log2 rho) - 53),
    r = max_l x_l; the proof of Lemma 2 places s_l1 on this grid and uses
    x_l - s_l1 >= 0;
  * P' = single_down( log2(P - 1) / 2 - 0.5 ).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache

import mpmath

from .fp import round_f32

# Section 3.1, eq. (p_list): the moduli fixed by the GEMMul8 library.
MODULI = (
    256, 255, 253, 251, 247, 241, 239, 233, 229, 227,
    223, 217, 211, 199, 197, 193, 191, 181, 179, 173,
    167, 163, 157, 151, 149, 139, 137, 131, 127, 113,
    109, 107, 103, 101, 97, 89, 83, 79, 73, 71,
    67, 61, 59, 53, 47, 43, 41, 37, 29,
)
N_MIN, N_MAX = 2, 49          # Algorithm 2/3 preconditions: 2 <= N <= 49
K_MAX = 2 ** 17               # Section 3: k <= 2^17
# Reading R22 (k beyond the paper's 2^17): every use of k <= 2^17 in
# Sections 3-4 is one of (i) Cbar = Abar Bbar <= 2^12 k exact in INT32,
# (ii) log2 Cbar <= 29 in the proofs of Lemmas 0 and 1, (iii) each residue
# product exact in INT32.  For k < 2^19, (i) still holds (2^12 k < 2^31),
# (ii) holds with 31 in place of 29 (the exhaustive claim of Lemma 0's proof
# can only fail for Cbar < 2^16, and Lemma 1's constant 147 u_32 becomes
# 157 u_32, still far inside its slack), and (iii) is kept by accumulating
# each residue product in chunks of 2^17 of k, each exact in INT32, whose
# residues mod p_l are added mod p_l.
K_MAX_EXT = 2 ** 19 - 1

U32 = Fraction(1, 2 ** 24)    # unit roundoff of FP32 (Section 1.2)
U64 = Fraction(1, 2 ** 53)    # unit roundoff of FP64


@dataclass(frozen=True)
class Constants:
    N: int
    b: int                  # 64 (DGEMM emulation) or 32 (SGEMM emulation)
    p: tuple                # moduli p_1..p_N
    P: int                  # product of the moduli
    q: tuple                # q_l = (P/p_l)^-1 mod p_l, 0 < q_l < p_l
    x: tuple                # x_l = (P/p_l) * q_l (exact integers)
    rho: int                # sum of floor(p_l / 2)
    clog2rho: int           # ceil(log2 rho)
    P1: float               # double(P)
    P2: float               # double(P - P1) for b=64, 0 for b=32
    Pinv: float             # double(1/P)
    s1: tuple               # s_l1 (FP64 values)
    s2: tuple               # s_l2 (FP64 values)
    s1_int: tuple           # s_l1 as exact integers (b=64); x_l rounded (b=32)
    Pprime: Fraction        # P' (an FP32 value)
    c: Fraction             # single_down(-0.5 / (1 - 4 u_32)), an FP32 value


def mpf_to_fraction(v) -> Fraction:
    """Exact rational value of an mpmath mpf."""
    man, exp = int(v.man), int(v.exp)
    return Fraction(man) * Fraction(2) ** exp


def c_constant() -> Fraction:
    """Algorithm 2, mu/nu steps: single_down(-0.5 / (1 - 4 u_32))."""
    return round_f32(Fraction(-1, 2) / (1 - 4 * U32), "rd")


def pprime(P: int) -> Fraction:
    """Algorithm 2, first step: P' = single_down(log2(P - 1)/2 - 0.5)."""
    with mpmath.workprec(256):
        v = mpmath.log(mpmath.mpf(P - 1), 2) / 2 - mpmath.mpf("0.5")
        vf = mpf_to_fraction(v)
    r = round_f32(vf, "rd")
    # The mpmath value is within ~2^-240 of the real one; the FP32 grid
    # spacing near v is >= 2^-21.  Require a wide margin on both sides so the
    # rounding cannot depend on the working precision.
    ulp = Fraction(2) ** (math.floor(math.log2(float(r))) - 23)
    margin = Fraction(1, 2 ** 200)
    assert vf - r > margin and (r + ulp) - vf > margin, "P' too close to the FP32 grid"
    return r


TABLES = ("paper", "optimal")


def moduli_for(N: int, table: str = "paper") -> tuple:
    """The N moduli: the first N of the fixed list of Section 3.1 ("paper"),
    or the N pairwise coprime moduli <= 256 of largest product ("optimal",
    the per-N tables Section 3.1 says can be built)."""
    if table == "paper":
        return MODULI[:N]
    if table == "optimal":
        from .moduli import optimal_moduli
        return optimal_moduli(N)
    raise ValueError(f"unknown moduli table {table!r}")


@lru_cache(maxsize=None)
def constants(N: int, b: int = 64, table: str = "paper") -> Constants:
    if not (N_MIN <= N <= N_MAX):
        raise ValueError(f"N must be in [{N_MIN}, {N_MAX}], got {N}")
    if b not in (32, 64):
        raise ValueError("b must be 32 or 64")
    p = moduli_for(N, table)
    P = math.prod(p)
    q = tuple(pow(P // pl, -1, pl) for pl in p)
    x = tuple((P // pl) * ql for pl, ql in zip(p, q))
    rho = sum(pl // 2 for pl in p)
    clog2rho = (rho - 1).bit_length()          # ceil(log2 rho) for rho >= 2
    P1 = float(P)                              # double(P): int->float is RN-even
    Pinv = 1 / P                               # int true division: RN of 1/P
    if b == 64:
        P2 = float(P - int(P1))
        r = max(x)
        gexp = r.bit_length() + clog2rho - 53  # floor(log2 r) + 1 + ceil(log2 rho) - 53
        if gexp <= 0:
            s1_int = x
        else:
            s1_int = tuple((xl >> gexp) << gexp for xl in x)
        s1 = tuple(float(v) for v in s1_int)
        assert all(int(a) == v for a, v in zip(s1, s1_int)), "s_l1 must be an FP64 value"
        s2 = tuple(float(xl - v) for xl, v in zip(x, s1_int))
    else:
        P2 = 0.0
        s1 = tuple(float(xl) for xl in x)      # s_l1 = double(x_l)
        s1_int = tuple(int(v) for v in s1)
        s2 = tuple(0.0 for _ in x)
    return Constants(N=N, b=b, p=p, P=P, q=q, x=x, rho=rho, clog2rho=clog2rho,
                     P1=P1, P2=P2, Pinv=Pinv, s1=s1, s2=s2, s1_int=s1_int,
                     Pprime=pprime(P), c=c_constant())


def beta(const: Constants) -> tuple:
    """beta_l of Section 3.1: number of upper bits of x_l kept in s_l1 (b=64)."""
    fr = max(const.x).bit_length() - 1
    return tuple(53 - const.clog2rho + (xl.bit_length() - 1) - fr for xl in const.x)
