// The real embedding of a complex product, written out (the complex planner
// ozaki2_zrequired_moduli runs the real planner on it; the GEMM calls form
// the embedding's slices in place instead):
//
//   Ahat = [[Ar, -Ai],      Bhat = [[Br],      Ahat Bhat = [[Re AB],
//           [Ai,  Ar]]              [Bi]]                   [Im AB]]
//
// The real Algorithm 1 runs unchanged on (Ahat, Bhat), so every quantity of
// Algorithms 1-3 and the Theorem 1 bound are those of the real 2m x n x 2k
// product.  The embedding kernels only move data: they write Ahat (2m x 2k)
// and Bhat (2k x n) column-major into the workspace from the interleaved
// (re, im) column-major inputs (the CRT writes the result as complex pairs).
// Indices run in 64-bit; threads walk consecutive rows, so every load and
// store of a wave is contiguous.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kMaxBlocks = 16384;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_embed_a(const T* __restrict__ A, int lda, int m,
                                                       int k, T* __restrict__ Ah) {
  const int64_t total = (int64_t)m * k, ldh = 2 * (int64_t)m;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kThreads) {
    const int64_t i = t % m, h = t / m;
    const T* a = A + 2 * (i + h * lda);
    const T re = a[0], im = a[1];
    T* c0 = Ah + h * ldh;              // column h:     [Ar; Ai]
    T* c1 = Ah + (h + k) * ldh;        // column k + h: [-Ai; Ar]
    c0[i] = re;
    c0[m + i] = im;
    c1[i] = -im;
    c1[m + i] = re;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_embed_b(const T* __restrict__ B, int ldb, int k,
                                                       int n, T* __restrict__ Bh) {
  const int64_t total = (int64_t)k * n, ldh = 2 * (int64_t)k;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kThreads) {
    const int64_t h = t % k, j = t / k;
    const T* b = B + 2 * (h + j * ldb);
    T* c = Bh + j * ldh;               // column j: [Br; Bi]
    c[h] = b[0];
    c[k + h] = b[1];
  }
}

dim3 grid_for(int64_t total) {
  const int64_t b = (total + kThreads - 1) / kThreads;
  return dim3((unsigned)(b < kMaxBlocks ? (b > 0 ? b : 1) : kMaxBlocks));
}

}  // namespace

void launch_embed_complex(hipStream_t s, Prec pr, const void* A, int lda, const void* B, int ldb,
                          int m, int n, int k, void* Ah, void* Bh) {
  const dim3 ga = grid_for((int64_t)m * k), gb = grid_for((int64_t)k * n), blk(kThreads);
  if (pr == Prec::F64) {
    hipLaunchKernelGGL(k_embed_a<double>, ga, blk, 0, s, (const double*)A, lda, m, k, (double*)Ah);
    hipLaunchKernelGGL(k_embed_b<double>, gb, blk, 0, s, (const double*)B, ldb, k, n, (double*)Bh);
  } else {
    hipLaunchKernelGGL(k_embed_a<float>, ga, blk, 0, s, (const float*)A, lda, m, k, (float*)Ah);
    hipLaunchKernelGGL(k_embed_b<float>, gb, blk, 0, s, (const float*)B, ldb, k, n, (float*)Bh);
  }
}

}  // namespace oz2
