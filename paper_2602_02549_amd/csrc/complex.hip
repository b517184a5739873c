// Complex GEMM through the real embedding (ozaki2_zgemm / ozaki2_cgemm):
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
#include "small_mod.h"

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

// ---- the 3-product form (ozaki2_zgemm3m) ---------------------------------
// Real and imaginary parts of an interleaved column-major matrix (rows x
// cols, leading dimension ld complex elements) as two planes with leading
// dimension `rows`.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_split(const T* __restrict__ X, int ld, int rows,
                                                     int cols, T* __restrict__ re,
                                                     T* __restrict__ im) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kThreads) {
    const int64_t i = t % rows, j = t / rows;
    const T* x = X + 2 * (i + j * ld);
    re[t] = x[0];
    im[t] = x[1];
  }
}

// Abar = (bar of the real part) + (bar of the imaginary part), each at most
// 32, as INT8 (count bytes, a multiple of 16).
__global__ __launch_bounds__(kThreads) void k_add_bars(const int8_t* __restrict__ a,
                                                        const int8_t* __restrict__ b,
                                                        int8_t* __restrict__ out, int64_t count) {
  const int64_t n16 = count / 16;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < n16;
       t += (int64_t)gridDim.x * kThreads) {
    const int4 x = reinterpret_cast<const int4*>(a)[t], y = reinterpret_cast<const int4*>(b)[t];
    // bytes in [0, 32]: lane-wise byte sums cannot carry into the next byte
    int4 r;
    r.x = x.x + y.x;
    r.y = x.y + y.y;
    r.z = x.z + y.z;
    r.w = x.w + y.w;
    reinterpret_cast<int4*>(out)[t] = r;
  }
}

// Residues of A'r + A'i: slice l of X3 = mod(X1 + X2, p_l), N slices of
// 16 * per16 bytes; workgroup row blockIdx.y is slice l, 16 bytes a thread.
__global__ __launch_bounds__(kThreads) void k_sum_residues(const int8_t* __restrict__ x1,
                                                            const int8_t* __restrict__ x2,
                                                            int8_t* __restrict__ x3, int64_t per16,
                                                            CrtConsts cc) {
  const int l = blockIdx.y;
  const SmallMod md(cc, l);
  const uint4* a = reinterpret_cast<const uint4*>(x1) + l * per16;
  const uint4* b = reinterpret_cast<const uint4*>(x2) + l * per16;
  uint4* c = reinterpret_cast<uint4*>(x3) + l * per16;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < per16;
       t += (int64_t)gridDim.x * kThreads) {
    const uint4 u = a[t], v = b[t];
    const uint32_t uw[4] = {u.x, u.y, u.z, u.w}, vw[4] = {v.x, v.y, v.z, v.w};
    uint32_t r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) r[q] |= md.byte(sbyte(uw[q], i) + sbyte(vw[q], i), i);
    }
    c[t] = make_uint4(r[0], r[1], r[2], r[3]);
  }
}

// W of the three products per modulus into the real and imaginary residues,
// in place: W1 <- mod(W1 - W2, p), W2 <- mod(W3 - W1 - W2, p) (layout as
// k_sum_residues).
__global__ __launch_bounds__(kThreads) void k_combine_w(int8_t* __restrict__ w1,
                                                         int8_t* __restrict__ w2,
                                                         const int8_t* __restrict__ w3,
                                                         int64_t per16, CrtConsts cc) {
  const int l = blockIdx.y;
  const SmallMod md(cc, l);
  uint4* a = reinterpret_cast<uint4*>(w1) + l * per16;
  uint4* b = reinterpret_cast<uint4*>(w2) + l * per16;
  const uint4* c = reinterpret_cast<const uint4*>(w3) + l * per16;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < per16;
       t += (int64_t)gridDim.x * kThreads) {
    const uint4 u = a[t], v = b[t], z = c[t];
    const uint32_t uw[4] = {u.x, u.y, u.z, u.w}, vw[4] = {v.x, v.y, v.z, v.w},
                   zw[4] = {z.x, z.y, z.z, z.w};
    uint32_t re[4], im[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      re[q] = 0;
      im[q] = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t1 = sbyte(uw[q], i), t2 = sbyte(vw[q], i), t3 = sbyte(zw[q], i);
        re[q] |= md.byte(t1 - t2, i);
        im[q] |= md.byte(t3 - t1 - t2, i);
      }
    }
    a[t] = make_uint4(re[0], re[1], re[2], re[3]);
    b[t] = make_uint4(im[0], im[1], im[2], im[3]);
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

void launch_split_complex(hipStream_t s, Prec pr, const void* X, int ld, int rows, int cols,
                          void* re, void* im) {
  const dim3 g = grid_for((int64_t)rows * cols), blk(kThreads);
  if (pr == Prec::F64)
    hipLaunchKernelGGL(k_split<double>, g, blk, 0, s, (const double*)X, ld, rows, cols, (double*)re,
                       (double*)im);
  else
    hipLaunchKernelGGL(k_split<float>, g, blk, 0, s, (const float*)X, ld, rows, cols, (float*)re,
                       (float*)im);
}

void launch_add_bars(hipStream_t s, const int8_t* a, const int8_t* b, int8_t* out, size_t count) {
  hipLaunchKernelGGL(k_add_bars, grid_for((int64_t)count / 16), dim3(kThreads), 0, s, a, b, out,
                     (int64_t)count);
}

// Grid of the slice-wise byte kernels: N rows of workgroups, each row
// covering one slice of per / 16 chunks (per is a multiple of 16: slices are
// padded to whole tiles).
dim3 byte_slice_grid(size_t per, int N) {
  const int64_t b = ((int64_t)(per / 16) + kThreads - 1) / kThreads;
  return dim3((unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024), (unsigned)N);
}

void launch_sum_residues(hipStream_t s, const int8_t* x1, const int8_t* x2, int8_t* x3, size_t per,
                         const CrtConsts& cc) {
  hipLaunchKernelGGL(k_sum_residues, byte_slice_grid(per, cc.N), dim3(kThreads), 0, s, x1, x2, x3,
                     (int64_t)(per / 16), cc);
}

void launch_combine_w(hipStream_t s, int8_t* w1, int8_t* w2, const int8_t* w3, size_t per,
                      const CrtConsts& cc) {
  hipLaunchKernelGGL(k_combine_w, byte_slice_grid(per, cc.N), dim3(kThreads), 0, s, w1, w2, w3,
                     (int64_t)(per / 16), cc);
}

}  // namespace oz2
