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
template <typename T, int R, bool DBG = false>
__device__ __forceinline__ void crt_body(const int8_t* __restrict__ W, size_t sw, int ldw,
                                const int* __restrict__ mu, const int* __restrict__ nu, int m,
                                int n, const CrtConsts& cc, const int* __restrict__ flag,
                                T* __restrict__ C, int ldc, int64_t g,
                                double* __restrict__ dbg = nullptr) {
  static_assert(R == 2 || R == 4 || R == 8, "rows per thread");
  typedef typename std::conditional<R == 2, uint16_t,
                                    typename std::conditional<R == 4, uint32_t, uint64_t>::type>::type
      WordT;
  const int chunks = cdiv_i(m, R);
  const int j = (int)(g / chunks);
  if (j >= n) return;
  const int i0 = (int)(g - (int64_t)j * chunks) * R;
  const int8_t* wp = W + (size_t)j * ldw + i0;
  double c1[R], c2[R];
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
    for (int u = 0; u < 4; ++u)
      wv[u] = *reinterpret_cast<const WordT*>(wp + (size_t)min(l0 + u, cc.N - 1) * sw);
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
  const bool bad = *flag != 0;
  const int nuj = nu[j];
  T out[R];
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const int i = min(i0 + e, m - 1);
    const double q = rint(c1[e] * cc.Pinv);
    const double t = fma(-q, cc.P1, c1[e]);
    const int ex = -mu[i] - nuj;
    double cppd;
    if (sizeof(T) == 8) {
      const double cpp = fma(-q, cc.P2, t + c2[e]);
      out[e] = bad ? (T)NAN : (T)ldexp(cpp, ex);
      cppd = cpp;
    } else {
      const float cpp = (float)t;
      out[e] = bad ? (T)NAN : (T)ldexp((double)cpp, ex);
      cppd = (double)cpp;
    }
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
