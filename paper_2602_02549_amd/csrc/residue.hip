// INT8 operand slices for the matrix-core products, written K-major
// (k contiguous per row of A, per column of B) and zero-padded to
// [rows_pad][k_pad]:
//   mode 0: Abar = ceil(diag(2^mu') |A|)            (Algorithm 2)
//   mode 1: A'_l = mod(trunc(diag(2^mu) A), p_l)     (Algorithms 2-3)
//
// A block stages a 64 x 64 tile of the FP64/FP32 source through LDS (so that
// both the column-major A and the column-major B are read coalesced), then
// each thread owns 16 consecutive k of one row and writes 16 bytes per slice.
//
// Residues of the scaled integer v = trunc(2^mu a) (|v| < 2^(6 + floor P'))
// are exact in FP64: each step r <- fma(-rint(r / p), p, r) is exact (the
// result is an integer of at most ~9 significant bits relative to ulp(q)),
// shrinks |r| by ~2^-52 relative, and the last step, taken with |r| < 2^50,
// lands in [-p/2, p/2] for odd p.  For p = 256 the INT8 cast wraps 128 to
// -128, which is congruent (Section 3.1).
#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr int kTile = 64;

__device__ inline int residue_i8(double v, int p, double pinv, int nsteps) {
  double r = v;
  for (int s = 0; s < nsteps; ++s) {
    double q = rint(r * pinv);
    r = fma(-q, (double)p, r);
  }
  int ri = (int)r;
  int half = p >> 1;
  if (ri > half) ri -= p;
  if (ri < -half) ri += p;
  return ri;  // p = 256: 128 stays 128 and is wrapped to -128 by the byte store
}

__device__ inline uint32_t pack4(int a, int b, int c, int d) {
  return (uint32_t)(a & 0xFF) | ((uint32_t)(b & 0xFF) << 8) | ((uint32_t)(c & 0xFF) << 16) |
         ((uint32_t)(d & 0xFF) << 24);
}

template <typename T, bool TRANS, int MODE>
__global__ __launch_bounds__(256) void k_slices(const T* __restrict__ src, int ld, int rows, int k,
                                                int k_pad, size_t slice, const uint64_t* __restrict__ bits,
                                                const int* __restrict__ shift, CrtConsts cc,
                                                int8_t* __restrict__ out) {
  __shared__ double tile[kTile][kTile + 1];
  const int t = threadIdx.x;
  const int r0 = blockIdx.y * kTile, h0 = blockIdx.x * kTile;
  if (TRANS) {  // src[r + h*ld]: consecutive threads take consecutive rows
    const int r = t & 63, rg = r0 + r;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int h = (t >> 6) + 4 * q, hg = h0 + h;
      tile[r][h] = (rg < rows && hg < k) ? (double)src[rg + (size_t)hg * ld] : 0.0;
    }
  } else {      // src[h + r*ld]: consecutive threads take consecutive k
    const int h = t & 63, hg = h0 + h;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = (t >> 6) + 4 * q, rg = r0 + r;
      tile[r][h] = (rg < rows && hg < k) ? (double)src[hg + (size_t)rg * ld] : 0.0;
    }
  }
  __syncthreads();

  const int r = t >> 2, hc = (t & 3) * 16, rg = r0 + r;
  double v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = tile[r][hc + e];
  int8_t* dst = out + (size_t)rg * k_pad + h0 + hc;

  if (MODE == 0) {
    const int sh = rg < rows ? shift_prime_bits(bits[rg]) : 0;
    int b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double x = fabs(v[e]);
      double c = ceil(ldexp(x, sh));
      b[e] = x == 0.0 ? 0 : (c < 1.0 ? 1 : (int)c);
    }
    uint4 w;
    w.x = pack4(b[0], b[1], b[2], b[3]);
    w.y = pack4(b[4], b[5], b[6], b[7]);
    w.z = pack4(b[8], b[9], b[10], b[11]);
    w.w = pack4(b[12], b[13], b[14], b[15]);
    *reinterpret_cast<uint4*>(dst) = w;
  } else {
    const int sh = rg < rows ? shift[rg] : 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = trunc(ldexp(v[e], sh));
    for (int l = 0; l < cc.N; ++l) {
      const int p = cc.p[l];
      const double pinv = cc.pinv[l];
      int b[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) b[e] = residue_i8(v[e], p, pinv, cc.nsteps);
      uint4 w;
      w.x = pack4(b[0], b[1], b[2], b[3]);
      w.y = pack4(b[4], b[5], b[6], b[7]);
      w.z = pack4(b[8], b[9], b[10], b[11]);
      w.w = pack4(b[12], b[13], b[14], b[15]);
      *reinterpret_cast<uint4*>(dst + (size_t)l * slice) = w;
    }
  }
}

template <typename T>
void launch_t(hipStream_t s, int mode, bool trans, const T* src, int ld, int rows, int k,
              int rows_pad, int k_pad, const uint64_t* bits, const int* shift, const CrtConsts& cc,
              int8_t* out) {
  dim3 grid(k_pad / kTile, rows_pad / kTile);
  size_t slice = (size_t)rows_pad * k_pad;
  if (mode == 0) {
    if (trans)
      hipLaunchKernelGGL((k_slices<T, true, 0>), grid, dim3(256), 0, s, src, ld, rows, k, k_pad,
                         slice, bits, shift, cc, out);
    else
      hipLaunchKernelGGL((k_slices<T, false, 0>), grid, dim3(256), 0, s, src, ld, rows, k, k_pad,
                         slice, bits, shift, cc, out);
  } else {
    if (trans)
      hipLaunchKernelGGL((k_slices<T, true, 1>), grid, dim3(256), 0, s, src, ld, rows, k, k_pad,
                         slice, bits, shift, cc, out);
    else
      hipLaunchKernelGGL((k_slices<T, false, 1>), grid, dim3(256), 0, s, src, ld, rows, k, k_pad,
                         slice, bits, shift, cc, out);
  }
}

}  // namespace

void launch_slices(hipStream_t s, Prec pr, int mode, bool trans, const void* src, int ld, int rows,
                   int k, int rows_pad, int k_pad, const uint64_t* bits, const int* shift,
                   const CrtConsts& cc, int8_t* out) {
  if (pr == Prec::F64)
    launch_t<double>(s, mode, trans, (const double*)src, ld, rows, k, rows_pad, k_pad, bits, shift,
                     cc, out);
  else
    launch_t<float>(s, mode, trans, (const float*)src, ld, rows, k, rows_pad, k_pad, bits, shift,
                    cc, out);
}

}  // namespace oz2
