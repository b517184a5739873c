// Scaling-vector kernels of Algorithm 2 (Section 3.2):
//   - per-row / per-column maximum of |a| (kept as the IEEE bit pattern of
//     the FP64 value, whose unsigned order equals the numeric order), from
//     which mu' = 5 - floor(log2 max|a|) follows exactly;
//   - the final shifts mu = mu' + floor(fma_down(c, e, P')) with
//     e = log2f(single_up(max_j Cbar_ij));
//   - log2f, correctly rounded to FP32 (double-double series evaluation).
#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr uint64_t kExpMask = 0x7FF0000000000000ull;

__device__ __forceinline__ void init_body(uint64_t* rowbits, int m_pad, uint64_t* colbits, int n_pad,
                                 int* rmax, int* cmax, int* flag, int t, int stride) {
  for (int i = t; i < m_pad; i += stride) {
    rowbits[i] = 0;
    rmax[i] = 0;
  }
  for (int j = t; j < n_pad; j += stride) {
    colbits[j] = 0;
    cmax[j] = 0;
  }
  if (t == 0) *flag = 0;
}

__global__ void k_init(uint64_t* rowbits, int m_pad, uint64_t* colbits, int n_pad, int* rmax,
                       int* cmax, int* flag) {
  init_body(rowbits, m_pad, colbits, n_pad, rmax, cmax, flag, blockIdx.x * blockDim.x + threadIdx.x,
            gridDim.x * blockDim.x);
}

// Bit pattern of |x| as FP64 (unsigned order = numeric order).
template <typename T>
__device__ __forceinline__ uint64_t abs_bits(T x) {
  return (uint64_t)__double_as_longlong(fabs((double)x));
}

// A column-major (m x k): one thread per row, a workgroup covers 256 rows and
// a chunk of 64 columns (workgroup bx + gx * by); consecutive threads read
// consecutive rows.  Loads go out 16 at a time from clamped (always valid)
// addresses; a repeated element does not change a maximum.  CX: A holds
// interleaved (re, im) pairs (lda in complex elements) and the maximum runs
// over both parts (the complex 3-product form's shared row shift).
template <typename T, bool CX = false>
__device__ __forceinline__ void absmax_rows_body(const T* __restrict__ A, int lda, int m, int k,
                                        uint64_t* __restrict__ rowbits, int* __restrict__ flag,
                                        int bx, int by, int dup = 0) {
  const int i = bx * 256 + threadIdx.x;
  constexpr int E = CX ? 2 : 1;   // T values per element
  const T* a = A + (size_t)E * min(i, m - 1);
  const int h0 = by * 64;
  uint64_t mx = 0;
#pragma unroll
  for (int q0 = 0; q0 < 64; q0 += 16) {
    T x[16], y[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const T* e = a + (size_t)E * ((size_t)min(h0 + q0 + u, k - 1) * lda);
      x[u] = e[0];
      if (CX) y[u] = e[1];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      uint64_t b = abs_bits(x[u]);
      if (CX) {
        const uint64_t c = abs_bits(y[u]);
        b = c > b ? c : b;
      }
      mx = b > mx ? b : mx;
    }
  }
  if (i >= m) return;
  if ((mx & kExpMask) == kExpMask) atomicOr(flag, 1);
  if (mx) {
    atomicMax((unsigned long long*)&rowbits[i], (unsigned long long)mx);
    // dup > 0: the same maximum for row i + dup (the two row blocks of the
    // real embedding of a complex matrix)
    if (dup) atomicMax((unsigned long long*)&rowbits[i + dup], (unsigned long long)mx);
  }
}

template <typename T, bool CX>
__global__ __launch_bounds__(256) void k_absmax_rows(const T* __restrict__ A, int lda, int m, int k,
                                                     uint64_t* __restrict__ rowbits,
                                                     int* __restrict__ flag, int dup) {
  const int gx = cdiv_i(m, 256);
  absmax_rows_body<T, CX>(A, lda, m, k, rowbits, flag, blockIdx.x % gx, blockIdx.x / gx, dup);
}

// B column-major (k x n): one wave per column j (four columns per
// workgroup), 16 loads in flight per lane; the wave owns the column and
// stores its maximum.  CX: interleaved (re, im) pairs, maximum over both
// parts, as for the rows.
template <typename T, bool CX = false>
__device__ __forceinline__ void absmax_cols_body(const T* __restrict__ B, int ldb, int k, int n,
                                        uint64_t* __restrict__ colbits, int* __restrict__ flag,
                                        int wg) {
  const int lane = threadIdx.x & 63;
  const int j = wg * 4 + (threadIdx.x >> 6);
  if (j >= n) return;   // whole wave
  constexpr int E = CX ? 2 : 1;
  const T* col = B + (size_t)E * ((size_t)j * ldb);
  uint64_t mx = 0;
  for (int h0 = 0; h0 < k; h0 += 1024) {
    T x[16], y[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const T* e = col + (size_t)E * min(h0 + lane + 64 * q, k - 1);
      x[q] = e[0];
      if (CX) y[q] = e[1];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      uint64_t b = abs_bits(x[q]);
      if (CX) {
        const uint64_t c = abs_bits(y[q]);
        b = c > b ? c : b;
      }
      mx = b > mx ? b : mx;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor((unsigned long long)mx, off);
    mx = o > mx ? o : mx;
  }
  if (lane == 0) {
    if ((mx & kExpMask) == kExpMask) atomicOr(flag, 1);
    colbits[j] = mx;
  }
}

template <typename T, bool CX>
__global__ __launch_bounds__(256) void k_absmax_cols(const T* __restrict__ B, int ldb, int k, int n,
                                                     uint64_t* __restrict__ colbits,
                                                     int* __restrict__ flag) {
  absmax_cols_body<T, CX>(B, ldb, k, n, colbits, flag, blockIdx.x);
}

// B column-major (k x n) with k_pad <= kAbsBarMaxK: the abs-max pass and the
// Bbar pass of Algorithm 2 in one read of B.  Each row j of the padded
// K-major Bbar (n_pad of them) is one column of B, held in registers (two
// consecutive k per lane, 32 per lane): a whole workgroup per column for
// k_pad > kAbsBarWaveK, one wave per column (four per workgroup) below.  The
// column's abs-max bit pattern is reduced over its threads, and
// Bbar = ceil(2^nu'_j |b|) (1 for a tiny nonzero b, 0 for b = 0) is written
// from the same registers, zero beyond k and for the padding rows j >= n.
constexpr int kAbsBarPasses = kAbsBarMaxK / 512;
static_assert(kAbsBarWaveK == kAbsBarPasses * 128, "a wave covers kAbsBarWaveK in the same passes");

__device__ __forceinline__ bool absbar_per_wave(int k_pad) { return k_pad <= kAbsBarWaveK; }

// Workgroups of absbar_cols_body for n_pad columns.
__host__ __device__ inline int absbar_blocks(int n_pad, int k_pad) {
  return k_pad <= kAbsBarWaveK ? (n_pad + 3) / 4 : n_pad;
}

template <typename T>
__device__ __forceinline__ void absbar_cols_body(const T* __restrict__ B, int ldb, int k, int n,
                                                 int n_pad, int k_pad,
                                                 uint64_t* __restrict__ colbits,
                                                 int* __restrict__ flag, int8_t* __restrict__ out,
                                                 int blk) {
  const bool per_wave = absbar_per_wave(k_pad);   // uniform over the launch
  const int tpc = per_wave ? 64 : 256;              // threads per column
  const int t = per_wave ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int j = per_wave ? blk * 4 + (int)(threadIdx.x >> 6) : blk;
  if (per_wave && j >= n_pad) return;               // whole wave; no barrier below for waves
  double x[2 * kAbsBarPasses];
  uint64_t mx = 0;
  if (j < n) {
    const T* col = B + (size_t)j * ldb;
#pragma unroll
    for (int q = 0; q < kAbsBarPasses; ++q) {
      const int h = 2 * t + 2 * tpc * q;
      x[2 * q] = h < k ? (double)col[h] : 0.0;
      x[2 * q + 1] = h + 1 < k ? (double)col[h + 1] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 2 * kAbsBarPasses; ++e) {
      const uint64_t b = (uint64_t)__double_as_longlong(fabs(x[e]));
      mx = b > mx ? b : mx;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 2 * kAbsBarPasses; ++e) x[e] = 0.0;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor((unsigned long long)mx, off);
    mx = o > mx ? o : mx;
  }
  if (!per_wave) {
    __shared__ unsigned long long red[4];
    if ((t & 63) == 0) red[t >> 6] = mx;
    __syncthreads();
    mx = red[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) mx = red[w] > mx ? red[w] : mx;
  }
  if (j < n && t == 0) {
    if ((mx & kExpMask) == kExpMask) atomicOr(flag, 1);
    colbits[j] = mx;
  }
  const int sh = j < n ? shift_prime_bits(mx) : 0;
  int8_t* dst = out + (size_t)j * k_pad;
#pragma unroll
  for (int q = 0; q < kAbsBarPasses; ++q) {
    const int h = 2 * t + 2 * tpc * q;
    if (h < k_pad) {
      int b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double a = fabs(x[2 * q + u]);
        const double cl = ceil(ldexp(a, sh));
        b[u] = a == 0.0 ? 0 : (cl < 1.0 ? 1 : (int)cl);
      }
      *reinterpret_cast<uint16_t*>(dst + h) = (uint16_t)((b[0] & 0xFF) | ((b[1] & 0xFF) << 8));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_absbar_cols(const T* __restrict__ B, int ldb, int k, int n,
                                                     int n_pad, int k_pad,
                                                     uint64_t* __restrict__ colbits,
                                                     int* __restrict__ flag,
                                                     int8_t* __restrict__ out) {
  absbar_cols_body<T>(B, ldb, k, n, n_pad, k_pad, colbits, flag, out, blockIdx.x);
}

// ---------------------------------------------------------------------------
// double-double helpers (Dekker / Knuth error-free transformations)
// ---------------------------------------------------------------------------
struct dd {
  double h, l;
};
__device__ inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd fast_two_sum(double a, double b) {  // |a| >= |b|
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.h, b.h);
  double e = s.l + (a.l + b.l);
  return fast_two_sum(s.h, e);
}
__device__ inline dd dd_mul(dd a, dd b) {
  double p = a.h * b.h;
  double e = fma(a.h, b.h, -p);
  e = fma(a.h, b.l, e);
  e = fma(a.l, b.h, e);
  return fast_two_sum(p, e);
}
__device__ inline dd dd_recip_int(int q) {  // 1/q as a double-double
  double h = 1.0 / (double)q;
  double r = fma(-h, (double)q, 1.0);      // exact remainder
  return {h, r / (double)q};
}

// log2 of an integer-valued d in [1, 2^30), rounded to nearest FP32.
// d = 2^E m with m in (1/sqrt2, sqrt2]; ln m = 2 atanh(z), z = (m-1)/(m+1),
// |z| <= 0.1716, summed to 23 terms in double-double (error < 2^-100), then
// multiplied by 1/ln2 (double-double constant).  The FP32 rounding of a
// double-double h + l is RN(h) unless h is exactly an FP32 midpoint, in which
// case the sign of l decides.
__device__ float log2f_rn(float dval) {
  double d = (double)dval;
  int E = ilogb(d);
  double mnt = ldexp(d, -E);
  if (mnt > 1.4142135623730951) {
    mnt *= 0.5;
    E += 1;
  }
  double num = mnt - 1.0;   // exact: mnt has at most 31 significant bits
  double den = mnt + 1.0;   // exact
  double zh = num / den;
  double zl = fma(-zh, den, num) / den;
  dd z = {zh, zl};
  dd z2 = dd_mul(z, z);
  dd T = dd_recip_int(2 * 22 + 1);
  for (int j = 21; j >= 0; --j) T = dd_add(dd_recip_int(2 * j + 1), dd_mul(z2, T));
  dd ln = dd_mul(z, T);
  ln.h *= 2.0;
  ln.l *= 2.0;
  const dd log2e = {0x1.71547652b82fep+0, 0x1.777d0ffda0d24p-56};
  dd r = dd_add(dd_mul(ln, log2e), dd{(double)E, 0.0});
  float y = (float)r.h;
  float yu = nextafterf(y, INFINITY), yd = nextafterf(y, -INFINITY);
  double mid_up = 0.5 * ((double)y + (double)yu), mid_dn = 0.5 * ((double)y + (double)yd);
  if (r.h == mid_up && r.l > 0) return yu;
  if (r.h == mid_dn && r.l < 0) return yd;
  return y;
}

// single_up of a nonnegative integer M <= 2^29 (exact below 2^24).
__device__ inline float single_up_int(int M) {
  unsigned u = (unsigned)M;
  int bl = 32 - __clz(u);
  if (bl > 24) {
    int s = bl - 24;
    u = ((u + (1u << s) - 1u) >> s) << s;
  }
  return (float)u;
}

// floor(c e + P') of the exact value: the product of two FP32 numbers is
// exact in FP64, and TwoSum gives the sum exactly as s + err; only an integer
// s with err < 0 needs a correction.
__device__ inline int floor_fma(float c, float e, float Pp) {
  double ce = (double)c * (double)e;
  dd s = two_sum(ce, (double)Pp);
  double f = floor(s.h);
  if (f == s.h && s.l < 0) f -= 1.0;
  return (int)f;
}

__device__ __forceinline__ void shifts_body(const uint64_t* __restrict__ rowbits, const int* __restrict__ rmax,
                                   int m, const uint64_t* __restrict__ colbits,
                                   const int* __restrict__ cmax, int n, float Pprime, float c,
                                   int* __restrict__ mu_p, int* __restrict__ nu_p,
                                   int* __restrict__ mu, int* __restrict__ nu,
                                   float* __restrict__ ef, int t, int bias = 0) {
  if (t >= m + n) return;
  const bool row = t < m;
  const int idx = row ? t : t - m;
  const uint64_t bits = row ? rowbits[idx] : colbits[idx];
  const int M = row ? rmax[idx] : cmax[idx];
  const int sp = shift_prime_bits(bits) + (bits ? bias : 0);
  const float d = single_up_int(M > 1 ? M : 1);       // R7: a zero maximum is treated as 1
  const float e = log2f_rn(d);
  const int s = sp + floor_fma(c, e, Pprime);
  if (row) {
    if (mu_p) mu_p[idx] = sp;
    mu[idx] = s;
  } else {
    if (nu_p) nu_p[idx] = sp;
    nu[idx] = s;
  }
  if (ef) ef[t] = e;
}

__global__ __launch_bounds__(256) void k_shifts(const uint64_t* __restrict__ rowbits,
                                                const int* __restrict__ rmax, int m,
                                                const uint64_t* __restrict__ colbits,
                                                const int* __restrict__ cmax, int n, float Pprime,
                                                float c, int* __restrict__ mu_p,
                                                int* __restrict__ nu_p, int* __restrict__ mu,
                                                int* __restrict__ nu, float* __restrict__ ef,
                                                int bias) {
  shifts_body(rowbits, rmax, m, colbits, cmax, n, Pprime, c, mu_p, nu_p, mu, nu, ef,
              blockIdx.x * 256 + threadIdx.x, bias);
}

// ---- grouped versions ------------------------------------------------------
__global__ __launch_bounds__(256) void kg_init(const ProbDesc* __restrict__ P,
                                               const BlockRef* __restrict__ map) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  init_body(d.rowbits, d.mp, d.colbits, d.np, d.rmax, d.cmax, d.flag, e.y * 256 + threadIdx.x,
            group_init_blocks(d.mp, d.np) * 256);
}

template <typename T>
__global__ __launch_bounds__(256) void kg_absmax_rows(const ProbDesc* __restrict__ P,
                                                      const BlockRef* __restrict__ map) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  const int gx = cdiv_i(d.m, 256);
  absmax_rows_body<T>((const T*)d.A, d.lda, d.m, d.k, d.rowbits, d.flag, e.y % gx, e.y / gx);
}

template <typename T>
__global__ __launch_bounds__(256) void kg_absmax_cols(const ProbDesc* __restrict__ P,
                                                      const BlockRef* __restrict__ map) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  absmax_cols_body<T>((const T*)d.B, d.ldb, d.k, d.n, d.colbits, d.flag, e.y);
}

// absbar_blocks(np, kp) workgroups per problem with k_pad <= kAbsBarMaxK.
template <typename T>
__global__ __launch_bounds__(256) void kg_absbar_cols(const ProbDesc* __restrict__ P,
                                                      const BlockRef* __restrict__ map) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  absbar_cols_body<T>((const T*)d.B, d.ldb, d.k, d.n, d.np, d.kp, d.colbits, d.flag, d.Bs, e.y);
}

__global__ __launch_bounds__(256) void kg_shifts(const ProbDesc* __restrict__ P,
                                                 const BlockRef* __restrict__ map,
                                                 const CrtConsts* __restrict__ ctab) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  const CrtConsts& cc = ctab[d.N];
  shifts_body(d.rowbits, d.rmax, d.m, d.colbits, d.cmax, d.n, cc.Pprime, cc.c, nullptr, nullptr,
              d.mu, d.nu, nullptr, e.y * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_log2f(const float* __restrict__ d, float* __restrict__ out,
                                               int count) {
  int t = blockIdx.x * 256 + threadIdx.x;
  if (t < count) out[t] = log2f_rn(d[t]);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace

void launch_init(hipStream_t s, uint64_t* rowbits, int m_pad, uint64_t* colbits, int n_pad,
                 int* rmax, int* cmax, int* flag) {
  int mx = m_pad > n_pad ? m_pad : n_pad;
  int blocks = cdiv(mx, 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, rowbits, m_pad, colbits, n_pad, rmax,
                     cmax, flag);
}

template <typename T, bool CX>
void absmax_rows_t(hipStream_t s, const void* A, int lda, int m, int k, uint64_t* rowbits,
                   int* flag, int dup) {
  const dim3 grid((unsigned)(cdiv(m, 256) * cdiv(k, 64)));
  hipLaunchKernelGGL((k_absmax_rows<T, CX>), grid, dim3(256), 0, s, (const T*)A, lda, m, k,
                     rowbits, flag, dup);
}

template <typename T, bool CX>
void absmax_cols_t(hipStream_t s, const void* B, int ldb, int k, int n, uint64_t* colbits,
                   int* flag) {
  const dim3 grid((unsigned)absmax_cols_blocks(n));
  hipLaunchKernelGGL((k_absmax_cols<T, CX>), grid, dim3(256), 0, s, (const T*)B, ldb, k, n,
                     colbits, flag);
}

void launch_absmax_rows(hipStream_t s, Prec pr, const void* A, int lda, int m, int k,
                        uint64_t* rowbits, int* flag, bool cx, int dup) {
  if (pr == Prec::F64)
    cx ? absmax_rows_t<double, true>(s, A, lda, m, k, rowbits, flag, dup)
       : absmax_rows_t<double, false>(s, A, lda, m, k, rowbits, flag, dup);
  else
    cx ? absmax_rows_t<float, true>(s, A, lda, m, k, rowbits, flag, dup)
       : absmax_rows_t<float, false>(s, A, lda, m, k, rowbits, flag, dup);
}

void launch_absmax_cols(hipStream_t s, Prec pr, const void* B, int ldb, int k, int n,
                        uint64_t* colbits, int* flag, bool cx) {
  if (pr == Prec::F64)
    cx ? absmax_cols_t<double, true>(s, B, ldb, k, n, colbits, flag)
       : absmax_cols_t<double, false>(s, B, ldb, k, n, colbits, flag);
  else
    cx ? absmax_cols_t<float, true>(s, B, ldb, k, n, colbits, flag)
       : absmax_cols_t<float, false>(s, B, ldb, k, n, colbits, flag);
}

int absbar_group_blocks(int n_pad, int k_pad) { return absbar_blocks(n_pad, k_pad); }

void launch_absbar_cols(hipStream_t s, Prec pr, const void* B, int ldb, int k, int n, int n_pad,
                        int k_pad, uint64_t* colbits, int* flag, int8_t* out) {
  if (n_pad <= 0) return;
  const dim3 grid((unsigned)absbar_blocks(n_pad, k_pad));
  if (pr == Prec::F64)
    hipLaunchKernelGGL(k_absbar_cols<double>, grid, dim3(256), 0, s, (const double*)B, ldb, k, n,
                       n_pad, k_pad, colbits, flag, out);
  else
    hipLaunchKernelGGL(k_absbar_cols<float>, grid, dim3(256), 0, s, (const float*)B, ldb, k, n,
                       n_pad, k_pad, colbits, flag, out);
}

void launch_shifts(hipStream_t s, const uint64_t* rowbits, const int* rmax, int m,
                   const uint64_t* colbits, const int* cmax, int n, float Pprime, float c,
                   int* mu_p, int* nu_p, int* mu, int* nu, float* ef, int bias) {
  hipLaunchKernelGGL(k_shifts, dim3(cdiv(m + n, 256)), dim3(256), 0, s, rowbits, rmax, m, colbits,
                     cmax, n, Pprime, c, mu_p, nu_p, mu, nu, ef, bias);
}

void launch_log2f(hipStream_t s, const float* d, float* out, int count) {
  hipLaunchKernelGGL(k_log2f, dim3(cdiv(count, 256)), dim3(256), 0, s, d, out, count);
}

void launch_group_scale(hipStream_t s, Prec pr, int phase, const ProbDesc* P, const BlockRef* map,
                        int blocks, const CrtConsts* ctab) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  switch (phase) {
    case GP_INIT:
      hipLaunchKernelGGL(kg_init, g, b, 0, s, P, map);
      break;
    case GP_ABSMAX_A:
      if (pr == Prec::F64)
        hipLaunchKernelGGL(kg_absmax_rows<double>, g, b, 0, s, P, map);
      else
        hipLaunchKernelGGL(kg_absmax_rows<float>, g, b, 0, s, P, map);
      break;
    case GP_ABSMAX_B:
      if (pr == Prec::F64)
        hipLaunchKernelGGL(kg_absmax_cols<double>, g, b, 0, s, P, map);
      else
        hipLaunchKernelGGL(kg_absmax_cols<float>, g, b, 0, s, P, map);
      break;
    case GP_ABSBAR_B:
      if (pr == Prec::F64)
        hipLaunchKernelGGL(kg_absbar_cols<double>, g, b, 0, s, P, map);
      else
        hipLaunchKernelGGL(kg_absbar_cols<float>, g, b, 0, s, P, map);
      break;
    case GP_SHIFTS:
      hipLaunchKernelGGL(kg_shifts, g, b, 0, s, P, map, ctab);
      break;
    default:
      break;
  }
}

}  // namespace oz2
