// Host construction of the per-N constants of Section 3.1 (Determination of
// Constants) and of the planner coefficients of Theorem 1 / eq. (thm:err-2).
//
// Exact quantities (P, q_l, x_l = (P/p_l) q_l, s_l1, s_l2, P1, P2, P_inv) are
// built with a small fixed-width unsigned big integer and correct rounding
// to FP64; P' and the constant c use 64-bit-mantissa long double arithmetic
// followed by an explicit round-down to FP32 and a margin check.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

// Section 3.1, eq. (p_list): the moduli, descending, pairwise coprime.
constexpr int kPaperModuli[kMaxModuli] = {
    256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193, 191,
    181, 179, 173, 167, 163, 157, 151, 149, 139, 137, 131, 127, 113, 109, 107, 103, 101,
    97,  89,  83,  79,  73,  71,  67,  61,  59,  53,  47,  43,  41,  37,  29};

// Unsigned integer of up to 512 bits, little-endian 64-bit limbs.
struct Big {
  static constexpr int L = 8;
  uint64_t w[L];
  Big() { std::memset(w, 0, sizeof(w)); }
  explicit Big(uint64_t v) : Big() { w[0] = v; }
  int bitlen() const {
    for (int i = L - 1; i >= 0; --i)
      if (w[i]) return 64 * i + 64 - __builtin_clzll(w[i]);
    return 0;
  }
  bool bit(int i) const { return i >= 0 && i < 64 * L && ((w[i / 64] >> (i % 64)) & 1u); }
  bool any_below(int i) const {  // any bit set strictly below position i
    for (int b = 0; b < i && b < 64 * L; ++b)
      if (bit(b)) return true;
    return false;
  }
  void mul_small(uint64_t v) {
    unsigned __int128 carry = 0;
    for (int i = 0; i < L; ++i) {
      unsigned __int128 t = (unsigned __int128)w[i] * v + carry;
      w[i] = (uint64_t)t;
      carry = t >> 64;
    }
  }
  uint64_t div_small(uint64_t v) {  // in place, returns remainder
    unsigned __int128 rem = 0;
    for (int i = L - 1; i >= 0; --i) {
      unsigned __int128 cur = (rem << 64) | w[i];
      w[i] = (uint64_t)(cur / v);
      rem = cur % v;
    }
    return (uint64_t)rem;
  }
  Big shr(int s) const {
    Big r;
    int q = s / 64, b = s % 64;
    for (int i = 0; i + q < L; ++i) {
      uint64_t lo = w[i + q] >> b;
      uint64_t hi = (b && i + q + 1 < L) ? (w[i + q + 1] << (64 - b)) : 0;
      r.w[i] = lo | hi;
    }
    return r;
  }
  Big shl(int s) const {
    Big r;
    int q = s / 64, b = s % 64;
    for (int i = L - 1; i >= q; --i) {
      uint64_t hi = w[i - q] << b;
      uint64_t lo = (b && i - q - 1 >= 0) ? (w[i - q - 1] >> (64 - b)) : 0;
      r.w[i] = hi | lo;
    }
    return r;
  }
  static int cmp(const Big& a, const Big& b) {
    for (int i = L - 1; i >= 0; --i)
      if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
  }
  static Big sub(const Big& a, const Big& b) {  // requires a >= b
    Big r;
    uint64_t borrow = 0;
    for (int i = 0; i < L; ++i) {
      uint64_t t = a.w[i] - b.w[i] - borrow;
      borrow = (a.w[i] < b.w[i] || (a.w[i] == b.w[i] && borrow)) ? 1 : 0;
      r.w[i] = t;
    }
    return r;
  }
  // Nearest FP64 value (ties to even).
  double to_double() const {
    int n = bitlen();
    if (n <= 53) {
      double r = 0;
      for (int i = L - 1; i >= 0; --i) r = r * 18446744073709551616.0 + (double)w[i];
      return r;  // exact: fewer than 54 significant bits
    }
    int s = n - 53;
    uint64_t top = shr(s).w[0];  // 53 bits
    bool half = bit(s - 1);
    bool sticky = any_below(s - 1);
    if (half && (sticky || (top & 1u))) ++top;
    return std::ldexp((double)top, s);
  }
  // Exact value of a finite nonnegative integer-valued double.
  static Big from_double(double d) {
    int e;
    double f = std::frexp(d, &e);  // d = f 2^e
    uint64_t mant = (uint64_t)std::ldexp(f, 53);
    Big r(mant);
    return e >= 53 ? r.shl(e - 53) : r.shr(53 - e);
  }
  // Top 64 bits (as long double) and the exponent of their lowest bit.
  long double top64(int* shift) const {
    int n = bitlen();
    int s = n > 64 ? n - 64 : 0;
    *shift = s;
    return (long double)shr(s).w[0];
  }
};

int modinv(int a, int p) {  // inverse of a modulo p (gcd(a, p) = 1), in [1, p-1]
  int t = 0, nt = 1, r = p, nr = a % p;
  while (nr) {
    int q = r / nr, tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  return t < 0 ? t + p : t;
}

// ---------------------------------------------------------------------------
// Moduli of largest product for each N (Section 3.1: the set that maximises
// P depends on N, 255 leaving it beyond a small N, so a table per N can be
// built).  Sought: N pairwise coprime integers in [2, 256] of largest
// product.  Every v <= 256 is s * q with s 13-smooth and q = 1 or a prime
// >= 17 (two primes >= 17 already exceed 256).  Coprimality therefore means:
// the 13-smooth parts use disjoint sets of the primes 2..13, and each prime
// >= 17 occurs at most once.  A dynamic program over "groups" -- one per
// prime q >= 17 (choose at most one multiple q s <= 256) and one per
// 13-smooth v (take it or not) -- keeps, per (set of small primes used,
// count chosen), the largest product; that is exact, because the groups'
// choices interact only through the small-prime set.  Among sets of equal
// product the one whose descending sequence is lexicographically larger is
// kept (that order is preserved when the same moduli are added to both, so
// the per-state choice is the global one).
struct ModSet {
  Big prod;                 // 0: state not reached
  std::vector<int> desc;    // the moduli, descending
};

bool better(const Big& p, const std::vector<int>& d, const ModSet& cur) {
  const int c = Big::cmp(p, cur.prod);
  if (c != 0) return c > 0;
  return std::lexicographical_compare(cur.desc.begin(), cur.desc.end(), d.begin(), d.end());
}

constexpr int kSmallPrimes[6] = {2, 3, 5, 7, 11, 13};

// Bit mask of the primes 2..13 dividing v, and the cofactor left over.
int small_mask(int v, int* rest) {
  int mask = 0;
  for (int i = 0; i < 6; ++i)
    if (v % kSmallPrimes[i] == 0) {
      mask |= 1 << i;
      while (v % kSmallPrimes[i] == 0) v /= kSmallPrimes[i];
    }
  *rest = v;
  return mask;
}

struct OptimalTable {
  bool ok = false;
  int p[kMaxModuli + 1][kMaxModuli];   // p[N][0..N-1], descending
  OptimalTable() {
    // groups of alternatives: each a list of (value, small-prime mask)
    std::vector<std::vector<std::pair<int, int>>> groups;
    std::vector<std::pair<int, int>> by_prime[257];
    for (int v = 2; v <= 256; ++v) {
      int rest;
      const int mask = small_mask(v, &rest);
      if (rest == 1)
        groups.push_back({{v, mask}});          // 13-smooth: its own group
      else
        by_prime[rest].push_back({v, mask});    // rest is a prime >= 17
    }
    for (int q = 17; q <= 256; ++q)
      if (!by_prime[q].empty()) groups.push_back(by_prime[q]);
    // dp[mask][count]
    std::vector<ModSet> dp(64 * (kMaxModuli + 1));
    auto st = [&](int mask, int cnt) -> ModSet& { return dp[mask * (kMaxModuli + 1) + cnt]; };
    st(0, 0).prod = Big(1);
    for (const auto& g : groups) {
      std::vector<ModSet> next = dp;            // "choose none of the group"
      for (int mask = 0; mask < 64; ++mask)
        for (int cnt = 0; cnt < kMaxModuli; ++cnt) {
          const ModSet& cur = st(mask, cnt);
          if (cur.prod.bitlen() == 0) continue;
          for (const auto& opt : g) {
            if (mask & opt.second) continue;
            Big prod = cur.prod;
            prod.mul_small((uint64_t)opt.first);
            std::vector<int> d = cur.desc;
            d.insert(std::upper_bound(d.begin(), d.end(), opt.first, std::greater<int>()),
                     opt.first);
            ModSet& dst = next[(mask | opt.second) * (kMaxModuli + 1) + cnt + 1];
            if (better(prod, d, dst)) {
              dst.prod = prod;
              dst.desc = std::move(d);
            }
          }
        }
      dp.swap(next);
    }
    for (int N = 2; N <= kMaxModuli; ++N) {
      ModSet best;
      for (int mask = 0; mask < 64; ++mask) {
        const ModSet& c = st(mask, N);
        if (c.prod.bitlen() != 0 && better(c.prod, c.desc, best)) best = c;
      }
      if ((int)best.desc.size() != N) return;
      for (int l = 0; l < N; ++l) p[N][l] = best.desc[l];
    }
    ok = true;
  }
};

// Round a long double down to an FP32 value (normal range); also returns the
// distance to the two neighbouring grid points in *margin.
float single_down(long double v, long double* margin) {
  int e;
  std::frexp(v, &e);                              // |v| = f 2^e, f in [0.5, 1)
  long double scaled = std::ldexp(v, 24 - e);     // 24 significant bits above the point
  long double fl = std::floor(scaled);
  float r = (float)std::ldexp(fl, e - 24);
  if (margin) {
    long double ulp = std::ldexp((long double)1, e - 24);
    long double lo = v - (long double)r, hi = (long double)r + ulp - v;
    *margin = lo < hi ? lo : hi;
  }
  return r;
}

// RN(1/P) by correcting a first guess with exact midpoint comparisons.
double recip_rn(const Big& P, double guess) {
  double y = guess;
  for (int iter = 0; iter < 8; ++iter) {
    int e;
    double f = std::frexp(y, &e);                 // y = M 2^(e-53), M in [2^52, 2^53)
    uint64_t M = (uint64_t)std::ldexp(f, 53);
    int ee = e - 53;
    // 1/P < (2M+1) 2^(ee-1)   <=>  (2M+1) P > 2^(1-ee)
    Big hi = P;
    hi.mul_small(2 * M + 1);
    Big pow_hi = Big(1).shl(1 - ee);
    bool below_hi = Big::cmp(hi, pow_hi) > 0;
    // lower midpoint: (2M-1) 2^(ee-1), or (4M-1) 2^(ee-2) when M = 2^52
    Big lo = P;
    int lo_sh;
    if (M == (1ull << 52)) {
      lo.mul_small(4 * M - 1);
      lo_sh = 2 - ee;
    } else {
      lo.mul_small(2 * M - 1);
      lo_sh = 1 - ee;
    }
    Big pow_lo = Big(1).shl(lo_sh);
    bool above_lo = Big::cmp(lo, pow_lo) < 0;     // 1/P > lower midpoint
    if (below_hi && above_lo) return y;
    y = below_hi ? std::nextafter(y, 0.0) : std::nextafter(y, 1.0);
  }
  return NAN;
}

}  // namespace

bool moduli_of(int table, int N, int* p) {
  if (N < 2 || N > kMaxModuli) return false;
  if (table == kTablePaper) {
    for (int l = 0; l < N; ++l) p[l] = kPaperModuli[l];
    return true;
  }
  if (table != kTableOptimal) return false;
  static const OptimalTable opt;   // built once, on first use
  if (!opt.ok) return false;
  for (int l = 0; l < N; ++l) p[l] = opt.p[N][l];
  return true;
}

bool build_consts(int N, int b, int table, CrtConsts* out) {
  if (N < 2 || N > kMaxModuli || (b != 64 && b != 32)) return false;
  int kModuli[kMaxModuli];
  if (!moduli_of(table, N, kModuli)) return false;
  CrtConsts cc;
  std::memset(&cc, 0, sizeof(cc));
  cc.N = N;
  cc.b = b;
  cc.table = table;
  Big P(1);
  int rho = 0;
  for (int l = 0; l < N; ++l) {
    P.mul_small((uint64_t)kModuli[l]);
    rho += kModuli[l] / 2;
  }
  int clog2rho = 0;
  while ((1 << clog2rho) < rho) ++clog2rho;

  // x_l = (P / p_l) q_l with q_l the inverse of prod_{h != l} p_h modulo p_l.
  Big x[kMaxModuli];
  int rmax_bits = 0;
  for (int l = 0; l < N; ++l) {
    int pl = kModuli[l];
    int rest = 1;
    for (int h = 0; h < N; ++h)
      if (h != l) rest = (int)(((int64_t)rest * (kModuli[h] % pl)) % pl);
    int q = modinv(rest, pl);
    Big t = P;
    if (t.div_small((uint64_t)pl) != 0) return false;
    t.mul_small((uint64_t)q);
    x[l] = t;
    int bl = t.bitlen();
    if (bl > rmax_bits) rmax_bits = bl;
  }

  for (int l = 0; l < N; ++l) {
    cc.p[l] = kModuli[l];
    cc.pinv[l] = 1.0 / (double)kModuli[l];
    if (b == 64) {
      // s_l1: upper beta_l bits of x_l, i.e. truncation to the grid
      // 2^(floor(log2 r) + 1 + ceil(log2 rho) - 53); s_l2 = double(x_l - s_l1).
      int gexp = rmax_bits + clog2rho - 53;
      Big s1 = gexp > 0 ? x[l].shr(gexp).shl(gexp) : x[l];
      cc.s1[l] = s1.to_double();
      if (Big::cmp(Big::from_double(cc.s1[l]), s1) != 0) return false;  // must be exact
      cc.s2[l] = Big::sub(x[l], s1).to_double();
    } else {
      cc.s1[l] = x[l].to_double();
      cc.s2[l] = 0.0;
    }
  }

  cc.P1 = P.to_double();
  if (b == 64) {
    Big P1i = Big::from_double(cc.P1);
    cc.P2 = Big::cmp(P, P1i) >= 0 ? Big::sub(P, P1i).to_double() : -Big::sub(P1i, P).to_double();
  } else {
    cc.P2 = 0.0;
  }
  cc.Pinv = recip_rn(P, 1.0 / cc.P1);
  if (!(cc.Pinv > 0)) return false;

  // P' = single_down(log2(P - 1)/2 - 0.5), Algorithm 2.
  Big Pm1 = Big::sub(P, Big(1));
  int sh;
  long double top = Pm1.top64(&sh);
  long double lg = (long double)sh + std::log2(top);  // dropped low bits: < 2^-63 relative
  long double v = lg / 2 - 0.5L;
  long double margin;
  cc.Pprime = single_down(v, &margin);
  if (!(margin > std::ldexp((long double)1, -40))) return false;
  // c = single_down(-0.5 / (1 - 4 u_32)).
  long double cv = -0.5L / (1.0L - 4.0L * std::ldexp((long double)1, -24));
  cc.c = single_down(cv, nullptr);

  // Residue reduction steps: |A'| < 2^(6 + floor(P')); a step maps |r| <= R
  // to |r| <= 128 + R 2^-51.9 and the last one needs R < 2^50 to be exact.
  long double R = std::ldexp((long double)1, 6 + (int)std::floor((double)cc.Pprime));
  int steps = 1;
  while (R >= std::ldexp((long double)1, 50)) {
    R = 128.0L + R * std::ldexp((long double)1, -51);
    ++steps;
  }
  if (steps > 4) return false;   // the residue kernels instantiate 1..4 steps
  cc.nsteps = steps;
  // Limbs of |A'| < 2^B: two (split at 2^48) keep the per-modulus sum below
  // 2^50 for B <= 90, three (split at 2^80 and 2^40) for B <= 122; for
  // B <= 50 one reduction step is cheaper.
  const int B = 6 + (int)std::floor((double)cc.Pprime);
  cc.nlimbs = B <= 50 ? 0 : (B <= 90 ? 2 : (B <= 122 ? 3 : 0));
  *out = cc;
  return true;
}

bool build_plan_coef(int b, int table, PlanCoef* out) {
  std::memset(out, 0, sizeof(*out));
  const long double u64 = std::ldexp((long double)1, -53), u32 = std::ldexp((long double)1, -24);
  for (int N = 2; N <= kMaxModuli; ++N) {
    int kModuli[kMaxModuli];
    if (!moduli_of(table, N, kModuli)) return false;
    Big P(1);
    int rho = 0;
    for (int l = 0; l < N; ++l) {
      P.mul_small((uint64_t)kModuli[l]);
      rho += kModuli[l] / 2;
    }
    int clog2rho = 0;
    while ((1 << clog2rho) < rho) ++clog2rho;
    int sh;
    long double Pm1 = Big::sub(P, Big(1)).top64(&sh);
    Pm1 = std::ldexp(Pm1, sh);                        // P - 1 (relative error < 2^-63)
    long double PP = std::ldexp(P.top64(&sh), sh);    // P
    long double tt = 1.0L / (32.0L * Pm1);            // t^2 = 1 / (2^5 (P - 1))
    long double extra, rnd, rconst, rrel;
    if (b == 64) {
      // r_64 - (3/2) u P = (1 + 3u) 2^(1 + ceil(log2 rho)) (N + 2) u^2 rho P
      rconst = (1 + 3 * u64) * std::ldexp((long double)1, 1 + clog2rho) * (N + 2) * u64 * u64 *
               rho * PP;
      rrel = 3 * u64;
      rnd = 1.5L * u64 * PP * tt;
    } else {
      // r_32 - (1/2) u_32 P = (1 + u_32) (N + 2) u_64 rho P
      rconst = (1 + u32) * (N + 2) * u64 * rho * PP;
      rrel = u32;
      rnd = 0.5L * u32 * PP * tt;
    }
    extra = rconst * tt;
    // Round every coefficient up so that the bound stays an upper bound.
    out->tt[N] = std::nextafter((double)tt, INFINITY);
    out->t[N] = std::nextafter(std::sqrt((double)tt), INFINITY);
    out->extra[N] = std::nextafter((double)extra, INFINITY);
    out->rnd[N] = std::nextafter((double)rnd, INFINITY);
    // Lemma 4 in the form |A'B' - C''| <= R_const + R_rel |A'B'|: R_const, and
    // R_rel t^2 / (1 - R_rel), the coefficient of (|C''| + R_const) in est1.
    out->rconst[N] = std::nextafter((double)rconst, INFINITY);
    out->rel[N] = std::nextafter((double)(rrel * tt / (1 - rrel)), INFINITY);
  }
  return true;
}

}  // namespace oz2
