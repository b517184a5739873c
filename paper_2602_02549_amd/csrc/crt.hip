// CRT accumulation, final reduction and inverse scaling (Algorithm 3 from the
// weighted sums on, and the last step of Algorithm 1), fused in one pass over
// the N INT8 slices W_l:
//   C'(1) = fl(sum_l s_l1 W_l)      (exact for b = 64, Lemma 2)
//   C'(2) = fl(sum_l s_l2 W_l)      (fma chain in l order; b = 64 only)
//   Q     = round(fl(P_inv C'(1)))  (equals round(C'/P), Lemma 3)
//   C''   = fl(fma(-Q, P2, fma(-Q, P1, C'(1)) + C'(2)))   (b = 64)
//   C''   = single(fma(-Q, P1, C'(1)))                      (b = 32)
//   C     = C'' * 2^(-mu_i - nu_j), one rounding.
// Every operation is an explicit fma / single rounding (built with
// -ffp-contract=off), so the result is deterministic.
#include <cstdint>
#include <type_traits>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

// One thread handles R = kCrtRows consecutive rows i of one column j: one
// R-byte load per modulus (64 R contiguous bytes per wave) and, when C is
// aligned for it, 2-element vector stores.
// Thread g (g = 0 .. ceil(m/R) n - 1) takes row chunk g % ceil(m/R) of column
// g / ceil(m/R): consecutive threads walk down a column and continue in the
// next, so small-m problems keep every lane busy.
// With DBG, C'(1), C'(2), Q and C'' of every entry are also stored, as FP64
// column-major m x n arrays at dbg + s * m * n for s = 0..3 (stage dumps).
// C'(1) and C'(2) of R consecutive rows (wp: row i0 of column j of slice 0).
// ALIGNED: wp is a multiple of R bytes, so each slice's R bytes are one load;
// otherwise they are gathered byte by byte.
template <typename T, int R, bool ALIGNED = true>
__device__ __forceinline__ void crt_sums(const int8_t* __restrict__ wp, size_t sw,
                                         const CrtConsts& cc, double (&c1)[R], double (&c2)[R]) {
  typedef typename std::conditional<R == 2, uint16_t,
                                    typename std::conditional<R == 4, uint32_t, uint64_t>::type>::type
      WordT;
#pragma unroll
  for (int e = 0; e < R; ++e) c1[e] = c2[e] = 0.0;
  // Moduli in groups of 4, loads first (clamped to the last slice); a modulus
  // past N gets weight 0, and fma(0, w, c) = c, so the l-ordered fma chains
  // are unchanged.
  // An INT8 value w with stored byte b becomes a double without the convert
  // instruction: the bit pattern 0x43300000:(b ^ 0x80) is 2^52 + w + 128, and
  // subtracting 2^52 + 128 is exact.
  for (int l0 = 0; l0 < cc.N; l0 += 4) {
    uint64_t wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int8_t* src = wp + (size_t)min(l0 + u, cc.N - 1) * sw;
      if constexpr (ALIGNED) {
        wv[u] = *reinterpret_cast<const WordT*>(src);
      } else {
        wv[u] = 0;
#pragma unroll
        for (int e = 0; e < R; ++e) wv[u] |= (uint64_t)(uint8_t)src[e] << (8 * e);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int l = min(l0 + u, cc.N - 1);
      const bool in = l0 + u < cc.N;
      const double s1 = in ? cc.s1[l] : 0.0, s2 = in ? cc.s2[l] : 0.0;
      const uint64_t biased = wv[u] ^ 0x8080808080808080ull;
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const int byte = (int)((biased >> (8 * e)) & 0xFF);
        const double w = __hiloint2double(0x43300000, byte) - 4503599627370624.0;  // 2^52 + 128
        c1[e] = fma(s1, w, c1[e]);
        if (sizeof(T) == 8) c2[e] = fma(s2, w, c2[e]);
      }
    }
  }
}

// Q, C'' and the output 2^ex C'' (NaN when the non-finite flag is set) of
// one entry from its C'(1), C'(2).
template <typename T>
__device__ __forceinline__ T crt_value(double c1, double c2, const CrtConsts& cc, int ex, bool bad,
                                       double* q_out, double* cpp_out) {
  const double q = rint(c1 * cc.Pinv);
  const double t = fma(-q, cc.P1, c1);
  double cppd;
  T out;
  if (sizeof(T) == 8) {
    const double cpp = fma(-q, cc.P2, t + c2);
    out = bad ? (T)NAN : (T)ldexp(cpp, ex);
    cppd = cpp;
  } else {
    const float cpp = (float)t;
    out = bad ? (T)NAN : (T)ldexp((double)cpp, ex);
    cppd = (double)cpp;
  }
  *q_out = q;
  *cpp_out = cppd;
  return out;
}

template <typename T, int R, bool DBG = false>
__device__ __forceinline__ void crt_body(const int8_t* __restrict__ W, size_t sw, int ldw,
                                const int* __restrict__ mu, const int* __restrict__ nu, int m,
                                int n, const CrtConsts& cc, const int* __restrict__ flag,
                                T* __restrict__ C, int ldc, int64_t g,
                                double* __restrict__ dbg = nullptr) {
  static_assert(R == 2 || R == 4 || R == 8, "rows per thread");
  const int chunks = cdiv_i(m, R);
  const int j = (int)(g / chunks);
  if (j >= n) return;
  const int i0 = (int)(g - (int64_t)j * chunks) * R;
  double c1[R], c2[R];
  crt_sums<T, R>(W + (size_t)j * ldw + i0, sw, cc, c1, c2);
  const bool bad = *flag != 0;
  const int nuj = nu[j];
  T out[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int i = min(i0 + e, m - 1);
    double q, cppd;
    out[e] = crt_value<T>(c1[e], c2[e], cc, -mu[i] - nuj, bad, &q, &cppd);
    if constexpr (DBG) {
      if (i0 + e < m) {
        const size_t mn = (size_t)m * n, o = (size_t)j * m + i0 + e;
        dbg[o] = c1[e];
        dbg[mn + o] = c2[e];
        dbg[2 * mn + o] = q;
        dbg[3 * mn + o] = cppd;
      }
    }
  }
  T* cp = C + (size_t)j * ldc + i0;
  if (i0 + R <= m && ((uintptr_t)cp & (2 * sizeof(T) - 1)) == 0) {
#pragma unroll
    for (int e = 0; e < R; e += 2) {
      if (sizeof(T) == 8) {
        double2 v;
        v.x = (double)out[e];
        v.y = (double)out[e + 1];
        *reinterpret_cast<double2*>(cp + e) = v;
      } else {
        float2 v;
        v.x = (float)out[e];
        v.y = (float)out[e + 1];
        *reinterpret_cast<float2*>(cp + e) = v;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (i0 + e < m) cp[e] = out[e];
  }
}

// Complex output: the real parts from (Wr, mur) and the imaginary parts from
// (Wi, mui), both with the column shifts nu, written as interleaved (re, im)
// pairs into the column-major complex C (ldc in complex elements).  The
// loads of a partial last chunk read up to row rup(m, R) - 1 past Wr and Wi,
// inside the padded column (the embedding's column holds 2m rows padded to a
// multiple of 128, at least m + rup(m, R)).
// R consecutive complex entries (rows i0.., column j) as interleaved pairs,
// with 2-element vector stores when the address allows.
template <typename T, int R>
__device__ __forceinline__ void store_complex(T* __restrict__ C, int ldc, int j, int i0, int m,
                                              const T (&re)[R], const T (&im)[R]) {
  T* cp = C + 2 * ((size_t)j * ldc + i0);
  if (i0 + R <= m && ((uintptr_t)cp & (2 * sizeof(T) - 1)) == 0) {
#pragma unroll
    for (int e = 0; e < R; ++e) {
      if (sizeof(T) == 8) {
        double2 v;
        v.x = (double)re[e];
        v.y = (double)im[e];
        *reinterpret_cast<double2*>(cp + 2 * e) = v;
      } else {
        float2 v;
        v.x = (float)re[e];
        v.y = (float)im[e];
        *reinterpret_cast<float2*>(cp + 2 * e) = v;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (i0 + e < m) {
        cp[2 * e] = re[e];
        cp[2 * e + 1] = im[e];
      }
  }
}

template <typename T, int R>
__device__ __forceinline__ void crt_complex_body(const int8_t* __restrict__ Wr,
                                                 const int8_t* __restrict__ Wi, size_t sw, int ldw,
                                                 const int* __restrict__ mur,
                                                 const int* __restrict__ mui,
                                                 const int* __restrict__ nu, int m, int n,
                                                 const CrtConsts& cc, const int* __restrict__ flag,
                                                 T* __restrict__ C, int ldc, int64_t g) {
  const int chunks = cdiv_i(m, R);
  const int j = (int)(g / chunks);
  if (j >= n) return;
  const int i0 = (int)(g - (int64_t)j * chunks) * R;
  const bool bad = *flag != 0;
  const int nuj = nu[j];
  double c1[R], c2[R], q, cppd;
  T re[R], im[R];
  crt_sums<T, R>(Wr + (size_t)j * ldw + i0, sw, cc, c1, c2);
#pragma unroll
  for (int e = 0; e < R; ++e)
    re[e] = crt_value<T>(c1[e], c2[e], cc, -mur[min(i0 + e, m - 1)] - nuj, bad, &q, &cppd);
  // the imaginary rows of the real embedding start at row m, which need not
  // be a multiple of R (uniform over the launch)
  if (((uintptr_t)Wi & (R - 1)) == 0)
    crt_sums<T, R, true>(Wi + (size_t)j * ldw + i0, sw, cc, c1, c2);
  else
    crt_sums<T, R, false>(Wi + (size_t)j * ldw + i0, sw, cc, c1, c2);
#pragma unroll
  for (int e = 0; e < R; ++e)
    im[e] = crt_value<T>(c1[e], c2[e], cc, -mui[min(i0 + e, m - 1)] - nuj, bad, &q, &cppd);
  store_complex<T, R>(C, ldc, j, i0, m, re, im);
}

// The 3-product form (reading R25 of the complex GEMM): per modulus l the
// real and imaginary residues are mod(W1 - W2, p_l) and mod(W3 - W1 - W2,
// p_l) of the three products' bytes, formed here and summed into C'(1),
// C'(2) of both parts with the l-ordered fma chains of crt_sums.  The bytes
// lie in [lo, hi] = [(1-p)/2, (p-1)/2] (odd p) or [-128, 127] (p = 256), so
// a difference or sum of two lies in [-(p-1), p-1] and one correction by p
// brings it back into [lo, hi]: W1 - W2 directly, W3 - W1 - W2 as W3 minus
// the corrected W1 + W2.  Moduli in groups of 4, loads first; a modulus past
// N gets weight 0 (fma(0, w, c) = c).  W1, W2, W3 are whole planes
// (tile-aligned), so each R-byte load is aligned.
template <typename T, int R>
__device__ __forceinline__ void crt_sums_3m(const int8_t* __restrict__ w1,
                                            const int8_t* __restrict__ w2,
                                            const int8_t* __restrict__ w3, size_t sw,
                                            const CrtConsts& cc, double (&c1r)[R], double (&c2r)[R],
                                            double (&c1i)[R], double (&c2i)[R]) {
  typedef typename std::conditional<R == 2, uint16_t,
                                    typename std::conditional<R == 4, uint32_t, uint64_t>::type>::type
      WordT;
#pragma unroll
  for (int e = 0; e < R; ++e) c1r[e] = c2r[e] = c1i[e] = c2i[e] = 0.0;
  for (int l0 = 0; l0 < cc.N; l0 += 4) {
    uint64_t a[4], b[4], c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t off = (size_t)min(l0 + u, cc.N - 1) * sw;
      a[u] = *reinterpret_cast<const WordT*>(w1 + off);
      b[u] = *reinterpret_cast<const WordT*>(w2 + off);
      c[u] = *reinterpret_cast<const WordT*>(w3 + off);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int l = min(l0 + u, cc.N - 1);
      const bool in = l0 + u < cc.N;
      const double s1 = in ? cc.s1[l] : 0.0, s2 = in ? cc.s2[l] : 0.0;
      const int p = cc.p[l], hi = (p - 1) / 2, lo = hi + 1 - p;
      auto fix = [&](int x) {
        x -= x > hi ? p : 0;
        return x + (x < lo ? p : 0);
      };
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const int t1 = (int)(int8_t)(a[u] >> (8 * e)), t2 = (int)(int8_t)(b[u] >> (8 * e)),
                  t3 = (int)(int8_t)(c[u] >> (8 * e));
        // w in [-128, 127] becomes a double without the convert instruction,
        // as in crt_sums: 0x43300000:(w + 128) is 2^52 + w + 128
        const double wr =
            __hiloint2double(0x43300000, fix(t1 - t2) + 128) - 4503599627370624.0;
        const double wi =
            __hiloint2double(0x43300000, fix(t3 - fix(t1 + t2)) + 128) - 4503599627370624.0;
        c1r[e] = fma(s1, wr, c1r[e]);
        c1i[e] = fma(s1, wi, c1i[e]);
        if (sizeof(T) == 8) {
          c2r[e] = fma(s2, wr, c2r[e]);
          c2i[e] = fma(s2, wi, c2i[e]);
        }
      }
    }
  }
}

template <typename T, int R>
__device__ __forceinline__ void crt_3m_body(const int8_t* __restrict__ W1,
                                            const int8_t* __restrict__ W2,
                                            const int8_t* __restrict__ W3, size_t sw, int ldw,
                                            const int* __restrict__ mu, const int* __restrict__ nu,
                                            int m, int n, const CrtConsts& cc,
                                            const int* __restrict__ flag, T* __restrict__ C,
                                            int ldc, int64_t g) {
  const int chunks = cdiv_i(m, R);
  const int j = (int)(g / chunks);
  if (j >= n) return;
  const int i0 = (int)(g - (int64_t)j * chunks) * R;
  const bool bad = *flag != 0;
  const int nuj = nu[j];
  const size_t o = (size_t)j * ldw + i0;
  double c1r[R], c2r[R], c1i[R], c2i[R], q, cppd;
  crt_sums_3m<T, R>(W1 + o, W2 + o, W3 + o, sw, cc, c1r, c2r, c1i, c2i);
  T re[R], im[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int ex = -mu[min(i0 + e, m - 1)] - nuj;
    re[e] = crt_value<T>(c1r[e], c2r[e], cc, ex, bad, &q, &cppd);
    im[e] = crt_value<T>(c1i[e], c2i[e], cc, ex, bad, &q, &cppd);
  }
  store_complex<T, R>(C, ldc, j, i0, m, re, im);
}

template <typename T, int R>
__global__ __launch_bounds__(256) void k_crt_3m(const int8_t* __restrict__ W1,
                                                const int8_t* __restrict__ W2,
                                                const int8_t* __restrict__ W3, size_t sw, int ldw,
                                                const int* __restrict__ mu,
                                                const int* __restrict__ nu, int m, int n,
                                                CrtConsts cc, const int* __restrict__ flag,
                                                T* __restrict__ C, int ldc) {
  crt_3m_body<T, R>(W1, W2, W3, sw, ldw, mu, nu, m, n, cc, flag, C, ldc,
                    (int64_t)blockIdx.x * 256 + threadIdx.x);
}

template <typename T, int R>
__global__ __launch_bounds__(256) void k_crt_complex(
    const int8_t* __restrict__ Wr, const int8_t* __restrict__ Wi, size_t sw, int ldw,
    const int* __restrict__ mur, const int* __restrict__ mui, const int* __restrict__ nu, int m,
    int n, CrtConsts cc, const int* __restrict__ flag, T* __restrict__ C, int ldc) {
  crt_complex_body<T, R>(Wr, Wi, sw, ldw, mur, mui, nu, m, n, cc, flag, C, ldc,
                         (int64_t)blockIdx.x * 256 + threadIdx.x);
}

template <typename T, int R>
__global__ __launch_bounds__(256) void k_crt(const int8_t* __restrict__ W, size_t sw, int ldw,
                                             const int* __restrict__ mu, const int* __restrict__ nu,
                                             int m, int n, CrtConsts cc,
                                             const int* __restrict__ flag, T* __restrict__ C, int ldc) {
  crt_body<T, R>(W, sw, ldw, mu, nu, m, n, cc, flag, C, ldc,
                 (int64_t)blockIdx.x * 256 + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_crt_debug(const int8_t* __restrict__ W, size_t sw, int ldw,
                                                   const int* __restrict__ mu,
                                                   const int* __restrict__ nu, int m, int n,
                                                   CrtConsts cc, const int* __restrict__ flag,
                                                   T* __restrict__ C, int ldc,
                                                   double* __restrict__ dbg) {
  crt_body<T, kCrtRows, true>(W, sw, ldw, mu, nu, m, n, cc, flag, C, ldc,
                              (int64_t)blockIdx.x * 256 + threadIdx.x, dbg);
}

template <typename T>
__global__ __launch_bounds__(256) void kg_crt(const ProbDesc* __restrict__ P,
                                              const BlockRef* __restrict__ map,
                                              const CrtConsts* __restrict__ ctab) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  crt_body<T, kCrtRows>(d.W, (size_t)d.np * d.mp, d.mp, d.mu, d.nu, d.m, d.n, ctab[d.N], d.flag,
                        (T*)d.C, d.ldc, (int64_t)e.y * 256 + threadIdx.x);
}

// Any problem's non-finite flag sets the sticky status word.
__global__ __launch_bounds__(256) void kg_or_status(const ProbDesc* __restrict__ P, int count,
                                                    int* __restrict__ status) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < count && *P[p].flag) atomicOr(status, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_zero(T* __restrict__ C, int ldc, int m,
                                                   int iblocks) {
  const int j = blockIdx.x / iblocks;
  const int i = (blockIdx.x % iblocks) * 256 + threadIdx.x;
  if (i < m) C[i + (size_t)j * ldc] = (T)0;
}

__global__ void k_or_status(const int* __restrict__ flag, int* __restrict__ status) {
  if (threadIdx.x == 0 && *flag) atomicOr(status, 1);
}

}  // namespace

void launch_or_status(hipStream_t s, const int* flag, int* status) {
  hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, s, flag, status);
}

void launch_group_crt(hipStream_t s, Prec pr, const ProbDesc* P, const BlockRef* map, int blocks,
                      int count, const CrtConsts* ctab, int* status) {
  if (blocks > 0) {
    if (pr == Prec::F64)
      hipLaunchKernelGGL(kg_crt<double>, dim3((unsigned)blocks), dim3(256), 0, s, P, map, ctab);
    else
      hipLaunchKernelGGL(kg_crt<float>, dim3((unsigned)blocks), dim3(256), 0, s, P, map, ctab);
  }
  hipLaunchKernelGGL(kg_or_status, dim3((unsigned)cdiv_i(count, 256)), dim3(256), 0, s, P, count,
                     status);
}

namespace {

template <typename T>
void launch_crt_t(hipStream_t s, const int8_t* W, size_t sw, int ldw, const int* mu, const int* nu,
                  int m, int n, const CrtConsts& cc, const int* flag, void* C, int ldc) {
  hipLaunchKernelGGL((k_crt<T, kCrtRows>), dim3((unsigned)crt_blocks(m, n)), dim3(256), 0, s, W, sw,
                     ldw, mu, nu, m, n, cc, flag, (T*)C, ldc);
}

}  // namespace

void launch_crt(hipStream_t s, Prec pr, const int8_t* W, size_t sw, int ldw, const int* mu,
                const int* nu, int m, int n, const CrtConsts& cc, const int* flag, void* C,
                int ldc) {
  if (pr == Prec::F64)
    launch_crt_t<double>(s, W, sw, ldw, mu, nu, m, n, cc, flag, C, ldc);
  else
    launch_crt_t<float>(s, W, sw, ldw, mu, nu, m, n, cc, flag, C, ldc);
}

void launch_crt_3m(hipStream_t s, Prec pr, const int8_t* W1, const int8_t* W2, const int8_t* W3,
                   size_t sw, int ldw, const int* mu, const int* nu, int m, int n,
                   const CrtConsts& cc, const int* flag, void* C, int ldc) {
  const dim3 grid((unsigned)crt_blocks(m, n)), block(256);
  if (pr == Prec::F64)
    hipLaunchKernelGGL((k_crt_3m<double, kCrtRows>), grid, block, 0, s, W1, W2, W3, sw, ldw, mu, nu,
                       m, n, cc, flag, (double*)C, ldc);
  else
    hipLaunchKernelGGL((k_crt_3m<float, kCrtRows>), grid, block, 0, s, W1, W2, W3, sw, ldw, mu, nu,
                       m, n, cc, flag, (float*)C, ldc);
}

void launch_crt_complex(hipStream_t s, Prec pr, const int8_t* Wr, const int8_t* Wi, size_t sw,
                        int ldw, const int* mur, const int* mui, const int* nu, int m, int n,
                        const CrtConsts& cc, const int* flag, void* C, int ldc) {
  const dim3 grid((unsigned)crt_blocks(m, n)), block(256);
  if (pr == Prec::F64)
    hipLaunchKernelGGL((k_crt_complex<double, kCrtRows>), grid, block, 0, s, Wr, Wi, sw, ldw, mur,
                       mui, nu, m, n, cc, flag, (double*)C, ldc);
  else
    hipLaunchKernelGGL((k_crt_complex<float, kCrtRows>), grid, block, 0, s, Wr, Wi, sw, ldw, mur,
                       mui, nu, m, n, cc, flag, (float*)C, ldc);
}

void launch_crt_debug(hipStream_t s, Prec pr, const int8_t* W, size_t sw, int ldw, const int* mu,
                      const int* nu, int m, int n, const CrtConsts& cc, const int* flag, void* C,
                      int ldc, double* dbg) {
  const dim3 grid((unsigned)crt_blocks(m, n)), block(256);
  if (pr == Prec::F64)
    hipLaunchKernelGGL(k_crt_debug<double>, grid, block, 0, s, W, sw, ldw, mu, nu, m, n, cc, flag,
                       (double*)C, ldc, dbg);
  else
    hipLaunchKernelGGL(k_crt_debug<float>, grid, block, 0, s, W, sw, ldw, mu, nu, m, n, cc, flag,
                       (float*)C, ldc, dbg);
}

void launch_fill_zero(hipStream_t s, Prec pr, void* C, int ldc, int m, int n) {
  const int iblocks = (m + 255) / 256;
  dim3 grid((unsigned)iblocks * (unsigned)n);
  if (pr == Prec::F64)
    hipLaunchKernelGGL(k_fill_zero<double>, grid, dim3(256), 0, s, (double*)C, ldc, m, iblocks);
  else
    hipLaunchKernelGGL(k_fill_zero<float>, grid, dim3(256), 0, s, (float*)C, ldc, m, iblocks);
}

}  // namespace oz2
