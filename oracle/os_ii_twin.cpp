// Plain C++ twin of the Python oracle (oracle/ozaki2.py): Algorithms 1-3 of
// the paper step by step, with plain loops (OpenMP over rows or columns), for
// timing on all host cores and as a second implementation that the Python
// oracle is compared with stage by stage.
//
// TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): nothing in the product
// path loads it.  It shares no code with the HIP library.  The constants of
// Section 3.1 (moduli, s_l1, s_l2, P1, P2, P_inv, P', c) are inputs, taken
// from oracle/constants.py; this file implements the steps, not the tables.
//
// Matrices are row-major here (A is m x k, B is k x n, outputs m x n), FP64
// values (FP32 inputs widened exactly).  Every step follows the paper's
// notation and the same readings as the Python oracle:
//   R4  zero row/column: mu' = 0;           R5  Abar = max(1, ceil(.)) for a != 0
//   R6  log2f correctly rounded to nearest; R7  zero maximum of Cbar -> 1
//   R8  floor(c e + P') of the exact value; R10 mod(x, 256) maps 128 to -128
//   R11 C'(2) (and C'(1) for b = 32) as the fma chain over l = 1..N
//   R13 one ldexp by -(mu_i + nu_j), FP32 output rounded once
//   R22 k beyond 2^17: residue products in chunks of 2^17 of k, their
//       residues added mod p_l.
#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int64_t kChunk = 1 << 17;

// mu' = 5 - floor(log2 x) for x = max_h |a_ih| (frexp is exact), 0 for x = 0.
int shift_prime(double x) {
  if (x == 0.0) return 0;
  int e;
  std::frexp(x, &e);   // x = f 2^e, f in [0.5, 1): floor(log2 x) = e - 1
  return 6 - e;
}

// single_up of a nonnegative integer as an FP32 value (returned as double).
double single_up(int64_t M) {
  float f = (float)M;                       // round to nearest
  if ((double)f < (double)M) f = std::nextafter(f, INFINITY);
  return (double)f;
}

// R6: correctly rounded FP32 log2 of an integer-valued d >= 1.  log2l has a
// 64-bit significand and an error of about one unit there; the result is
// refused (NaN) if that value lies within 2^-56 (relative) of an FP32
// rounding midpoint, where the rounding could depend on that error.
double log2f_rn(double d) {
  const long double v = log2l((long double)d);
  const float r = (float)v;
  if (v == 0.0L) return 0.0;
  const long double up = (long double)std::nextafter(r, INFINITY);
  const long double dn = (long double)std::nextafter(r, -INFINITY);
  const long double mu = ((long double)r + up) / 2, md = ((long double)r + dn) / 2;
  const long double tol = fabsl(v) * 0x1p-56L;
  if (fabsl(v - mu) <= tol || fabsl(v - md) <= tol) return NAN;
  return (double)r;
}

// mod(x, p) in the symmetric INT8 range: x - p round(x / p), with the tie of
// p = 256 (x = 128 mod 256) mapped to -128.  fmod is exact.
int mod_sym(double x, int p) {
  double r = std::fmod(x, (double)p);         // exact, sign of x, |r| < p
  if (r < 0) r += p;                          // [0, p)
  if (r >= (p + 1) / 2) r -= p;               // odd p: (p/2, p) -> negative; 256: 128 -> -128
  return (int)r;
}

int mod_sym_int(int64_t x, int p) {
  int64_t r = x % p;
  if (r < 0) r += p;
  if (r >= (p + 1) / 2) r -= p;
  return (int)r;
}

int32_t wrap_int32(int64_t x) { return (int32_t)(uint32_t)(uint64_t)x; }

}  // namespace

extern "C" {

// Threads the OpenMP loops of the twin use.
int ozaki2_oracle_twin_threads(void) { return omp_get_max_threads(); }

// Outputs may be NULL where noted; C is required.  Returns 0, or -1 for an
// input outside the method's domain (non-finite), -2 if a log2f value could
// not be decided (see log2f_rn), -3 if Abar left [0, 64].
//   b       : 64 or 32 (output rounding of Algorithm 3's last step)
//   consts  : N moduli p (int), then doubles s1[N], s2[N], P1, P2, Pinv,
//             Pprime, c (passed separately below)
int ozaki2_oracle_twin(int b, int m, int n, int k, const double* A, const double* B, int N,
                       const int* p, const double* s1, const double* s2, double P1, double P2,
                       double Pinv, double Pprime, double c, int* mu_p_out, int* nu_p_out,
                       int64_t* rmax_out, int64_t* cmax_out, int* mu_out, int* nu_out,
                       int8_t* Al_out, int8_t* Bl_out, int8_t* W_out, double* C1_out,
                       double* C2_out, double* Q_out, double* Cpp_out, double* C) {
  const size_t mk = (size_t)m * k, kn = (size_t)k * n, mn = (size_t)m * n;
  for (size_t t = 0; t < mk; ++t)
    if (!std::isfinite(A[t])) return -1;
  for (size_t t = 0; t < kn; ++t)
    if (!std::isfinite(B[t])) return -1;

  // ---- Algorithm 2: mu', nu', Abar, Bbar ---------------------------------
  std::vector<int> mup(m), nup(n);
  for (int i = 0; i < m; ++i) {
    double x = 0;
    for (int h = 0; h < k; ++h) x = std::fmax(x, std::fabs(A[(size_t)i * k + h]));
    mup[i] = shift_prime(x);
  }
  for (int j = 0; j < n; ++j) {
    double x = 0;
    for (int h = 0; h < k; ++h) x = std::fmax(x, std::fabs(B[(size_t)h * n + j]));
    nup[j] = shift_prime(x);
  }
  std::vector<int16_t> Abar(mk), Bbar(kn);
  bool bad_bar = false;
#pragma omp parallel for reduction(|| : bad_bar)
  for (int i = 0; i < m; ++i)
    for (int h = 0; h < k; ++h) {
      const double a = std::fabs(A[(size_t)i * k + h]);
      double v = std::ceil(std::ldexp(a, mup[i]));
      if (a != 0 && v < 1) v = 1;
      if (v < 0 || v > 64) bad_bar = true;
      Abar[(size_t)i * k + h] = (int16_t)v;
    }
#pragma omp parallel for reduction(|| : bad_bar)
  for (int h = 0; h < k; ++h)
    for (int j = 0; j < n; ++j) {
      const double x = std::fabs(B[(size_t)h * n + j]);
      double v = std::ceil(std::ldexp(x, nup[j]));
      if (x != 0 && v < 1) v = 1;
      if (v < 0 || v > 64) bad_bar = true;
      Bbar[(size_t)h * n + j] = (int16_t)v;
    }
  if (bad_bar) return -3;

  // ---- Cbar = Abar Bbar (exact integers), row and column maxima ----------
  std::vector<int64_t> rmax(m, 0), cmax(n, 0);
#pragma omp parallel
  {
    std::vector<int64_t> cm(n, 0), row(n);
#pragma omp for
    for (int i = 0; i < m; ++i) {
      std::fill(row.begin(), row.end(), 0);
      for (int h = 0; h < k; ++h) {
        const int64_t a = Abar[(size_t)i * k + h];
        if (!a) continue;
        const int16_t* brow = &Bbar[(size_t)h * n];
        for (int j = 0; j < n; ++j) row[j] += a * brow[j];
      }
      int64_t mx = 0;
      for (int j = 0; j < n; ++j) {
        mx = row[j] > mx ? row[j] : mx;
        cm[j] = row[j] > cm[j] ? row[j] : cm[j];
      }
      rmax[i] = mx;
    }
#pragma omp critical
    for (int j = 0; j < n; ++j) cmax[j] = cm[j] > cmax[j] ? cm[j] : cmax[j];
  }

  // ---- Dbar, e, f, mu, nu ---------------------------------------------------
  std::vector<int> mu(m), nu(n);
  bool undecided = false;
  auto shift = [&](int sp, int64_t M) {
    const double d = single_up(M > 0 ? M : 1);            // R7
    const double e = log2f_rn(d);
    if (std::isnan(e)) undecided = true;
    // c e is exact in FP64 (two 24-bit significands); adding P' is exact in
    // the 64-bit significand of long double, so the floor is of the exact
    // value (R8).
    const long double x = (long double)(c * e) + (long double)Pprime;
    return sp + (int)floorl(x);
  };
  for (int i = 0; i < m; ++i) mu[i] = shift(mup[i], rmax[i]);
  for (int j = 0; j < n; ++j) nu[j] = shift(nup[j], cmax[j]);
  if (undecided) return -2;

  // ---- A' = trunc(2^mu A), B' = trunc(B 2^nu) (exact in FP64) ------------
  std::vector<double> Ap(mk), Bp(kn);
#pragma omp parallel for
  for (int i = 0; i < m; ++i)
    for (int h = 0; h < k; ++h) Ap[(size_t)i * k + h] = std::trunc(std::ldexp(A[(size_t)i * k + h], mu[i]));
#pragma omp parallel for
  for (int h = 0; h < k; ++h)
    for (int j = 0; j < n; ++j) Bp[(size_t)h * n + j] = std::trunc(std::ldexp(B[(size_t)h * n + j], nu[j]));

  // ---- Algorithm 3: residues, residue products, W ------------------------
  std::vector<int8_t> al(mk), bl(kn), W((size_t)N * mn);
  std::vector<int8_t> blT(kn);
  for (int l = 0; l < N; ++l) {
    const int pl = p[l];
#pragma omp parallel for
    for (int64_t t = 0; t < (int64_t)mk; ++t) al[t] = (int8_t)mod_sym(Ap[t], pl);
#pragma omp parallel for
    for (int64_t t = 0; t < (int64_t)kn; ++t) bl[t] = (int8_t)mod_sym(Bp[t], pl);
    if (Al_out) std::memcpy(Al_out + (size_t)l * mk, al.data(), mk);
    if (Bl_out) std::memcpy(Bl_out + (size_t)l * kn, bl.data(), kn);
    for (int h = 0; h < k; ++h)
      for (int j = 0; j < n; ++j) blT[(size_t)j * k + h] = bl[(size_t)h * n + j];
    int8_t* Wl = &W[(size_t)l * mn];
#pragma omp parallel for collapse(2)
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) {
        const int8_t* ar = &al[(size_t)i * k];
        const int8_t* bc = &blT[(size_t)j * k];
        int w = 0;
        for (int64_t h0 = 0; h0 < k; h0 += kChunk) {     // one INT32 product per chunk (R22)
          const int64_t h1 = h0 + kChunk < k ? h0 + kChunk : k;
          int64_t s = 0;
          for (int64_t h = h0; h < h1; ++h) s += (int32_t)ar[h] * (int32_t)bc[h];
          w = mod_sym_int((int64_t)w + mod_sym_int(wrap_int32(s), pl), pl);
        }
        Wl[(size_t)i * n + j] = (int8_t)w;
      }
  }
  if (W_out) std::memcpy(W_out, W.data(), (size_t)N * mn);

  // ---- C'(1), C'(2), Q, C'' and the inverse scaling ---------------------
#pragma omp parallel for
  for (int64_t t = 0; t < (int64_t)mn; ++t) {
    double c1 = 0, c2 = 0;
    for (int l = 0; l < N; ++l) {
      const double w = (double)W[(size_t)l * mn + t];
      if (b == 64) {
        c1 = c1 + s1[l] * w;              // exact (Lemma 2)
        c2 = std::fma(s2[l], w, c2);      // R11
      } else {
        c1 = std::fma(s1[l], w, c1);      // R11 for b = 32
      }
    }
    const double q = std::nearbyint(Pinv * c1);   // ties cannot occur (Lemma 3)
    const double tt = std::fma(-q, P1, c1);
    double cpp;
    if (b == 64)
      cpp = std::fma(-q, P2, tt + c2);
    else
      cpp = (double)(float)tt;
    const int i = (int)(t / n), j = (int)(t % n);
    const double out = std::ldexp(cpp, -mu[i] - nu[j]);
    C[t] = b == 64 ? out : (double)(float)out;
    if (C1_out) C1_out[t] = c1;
    if (C2_out) C2_out[t] = c2;
    if (Q_out) Q_out[t] = q;
    if (Cpp_out) Cpp_out[t] = cpp;
  }
  for (int i = 0; i < m; ++i) {
    if (mu_p_out) mu_p_out[i] = mup[i];
    if (rmax_out) rmax_out[i] = rmax[i];
    if (mu_out) mu_out[i] = mu[i];
  }
  for (int j = 0; j < n; ++j) {
    if (nu_p_out) nu_p_out[j] = nup[j];
    if (cmax_out) cmax_out[j] = cmax[j];
    if (nu_out) nu_out[j] = nu[j];
  }
  return 0;
}

}  // extern "C"
