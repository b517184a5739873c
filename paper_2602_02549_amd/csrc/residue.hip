// INT8 operand slices for the matrix-core products, written K-major
// (k contiguous per row of A, per column of B) and zero-padded to
// [rows_pad][k_pad]:
//   mode 0: Abar = ceil(diag(2^mu') |A|)            (Algorithm 2)
//   mode 1: A'_l = mod(trunc(diag(2^mu) A), p_l)     (Algorithms 2-3)
//
// A block stages a 32-row x 128-k tile of the FP64/FP32 source through LDS:
// the column-major A (rows contiguous) and the column-major B (k contiguous)
// are both read coalesced, then each thread owns 16 consecutive k of one row
// and writes 16 bytes per slice, 8 threads covering one full 128-byte line.
// The LDS rows are 132 doubles apart and their columns XOR-swizzled by
// (row / 8), and each thread walks its 16 elements starting at its chunk
// index: both the staging stores and the reads then touch every bank exactly
// twice per wave (the minimum for 64 x 8 bytes).
//
// Residues of the scaled integer v = trunc(2^mu a) (|v| < 2^(6 + floor P'))
// are exact in FP64.  Up to three 32-bit limbs (N <= 20): v = sum_t v_t 2^(32t)
// with |v_t| <= 2^31 below the top limb, split once per element; per modulus
// r = v_0 + sum_t v_t c_t with c_t = mod(2^(32t), p) (exact: |r| < 2^41), and
// one step r <- fma(-rint(r / p), p, r) lands in [-(p-1)/2, (p-1)/2] for odd
// p.  Larger N take nsteps such steps from v itself (each exact, shrinking |r|
// by ~2^-52 relative; the last starts from |r| < 2^50).  For p = 256 the
// result lies in [-128, 128] and the byte store wraps 128 to -128.
#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr int kTR = 32;           // slice tile: rows
constexpr int kTK = 128;          // slice tile: k
constexpr int kRS = kTK + 4;      // LDS row stride (doubles)
constexpr int kPlanTile = 64;     // planner operand tile

// nsteps reduction steps (the last from |r| < 2^50); NS = 1..4 for N <= 49.
template <int NS>
__device__ __forceinline__ int residue_i8(double v, int p, double pinv) {
  double r = v;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double q = rint(r * pinv);
    r = fma(-q, (double)p, r);
  }
  return (int)r;
}

__device__ inline uint32_t pack4(int a, int b, int c, int d) {
  return (uint32_t)(a & 0xFF) | ((uint32_t)(b & 0xFF) << 8) | ((uint32_t)(c & 0xFF) << 16) |
         ((uint32_t)(d & 0xFF) << 24);
}

// The N residue bytes of 16 consecutive k of one row, one 16-byte store per
// modulus.
template <int NS>
__device__ __forceinline__ void store_residues(const double (&v)[16], const CrtConsts& cc,
                                               int8_t* __restrict__ dst, size_t slice) {
  for (int l = 0; l < cc.N; ++l) {
    const int p = cc.p[l];
    const double pinv = cc.pinv[l];
    int b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) b[e] = residue_i8<NS>(v[e], p, pinv);
    uint4 w;
    w.x = pack4(b[0], b[1], b[2], b[3]);
    w.y = pack4(b[4], b[5], b[6], b[7]);
    w.z = pack4(b[8], b[9], b[10], b[11]);
    w.w = pack4(b[12], b[13], b[14], b[15]);
    *reinterpret_cast<uint4*>(dst + (size_t)l * slice) = w;
  }
}

// Limb form of the residues (L = 2 or 3 limbs of 32 bits).
__device__ __forceinline__ double reduce_once(double r, double p, double pinv) {
  return fma(-rint(r * pinv), p, r);
}

template <int L>
__device__ __forceinline__ void store_residues_limbs(const double (&v)[16], const CrtConsts& cc,
                                                     int8_t* __restrict__ dst, size_t slice) {
  static_assert(L == 2 || L == 3, "limbs");
  double lo[16], mid[16], hi[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    double rem = v[e];
    if (L == 3) {
      hi[e] = rint(rem * 0x1p-64);
      rem = fma(-hi[e], 0x1p64, rem);          // exact, |rem| <= 2^63
    }
    mid[e] = rint(rem * 0x1p-32);
    lo[e] = fma(-mid[e], 0x1p32, rem);         // exact, |lo| <= 2^31
  }
  for (int l = 0; l < cc.N; ++l) {
    const double p = (double)cc.p[l];
    const double pinv = cc.pinv[l];
    const double c1 = reduce_once(0x1p32, p, pinv);                 // mod(2^32, p)
    const double c2 = L == 3 ? reduce_once(c1 * c1, p, pinv) : 0.0;  // mod(2^64, p)
    int b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double r = fma(mid[e], c1, lo[e]);
      if (L == 3) r = fma(hi[e], c2, r);
      b[e] = (int)reduce_once(r, p, pinv);
    }
    uint4 w;
    w.x = pack4(b[0], b[1], b[2], b[3]);
    w.y = pack4(b[4], b[5], b[6], b[7]);
    w.z = pack4(b[8], b[9], b[10], b[11]);
    w.w = pack4(b[12], b[13], b[14], b[15]);
    *reinterpret_cast<uint4*>(dst + (size_t)l * slice) = w;
  }
}

// One 32-row x 128-k tile (k tile kx, row tile ry) of the slices.
template <typename T, bool TRANS, int MODE>
__device__ __forceinline__ void slices_body(const T* __restrict__ src, int ld, int rows, int k, int k_pad,
                                   size_t slice, const uint64_t* __restrict__ bits,
                                   const int* __restrict__ shift, const CrtConsts& cc,
                                   int8_t* __restrict__ out, int kx, int ry) {
  __shared__ double tile[kTR * kRS];
  const int t = threadIdx.x;
  const int r0 = ry * kTR, h0 = kx * kTK;
  // Residue slices of padding rows feed only products of padding rows, which
  // the CRT never reads: they are left unwritten (the k padding of real rows
  // is still zeroed).  Abar/Bbar padding must stay zero, since the scaling
  // product's maxima cover whole rows and columns.
  if (MODE == 1 && r0 >= rows) return;   // whole workgroup, before any barrier
  // All 16 loads of a thread go out before any is used: their addresses are
  // clamped into the matrix and out-of-range elements are replaced by zero
  // afterwards, so no branch separates them.
  T x[16];
  if (TRANS) {  // src[r + h*ld]: 32 consecutive rows per half-wave, two columns per wave
    const int r = t & 31, rg = r0 + r, sw = r >> 3;
    const int hb = t >> 5;
    const T* a = src + min(rg, rows - 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = a[(size_t)min(h0 + hb + 8 * q, k - 1) * ld];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int h = hb + 8 * q;
      tile[r * kRS + (h ^ sw)] = (rg < rows && h0 + h < k) ? (double)x[q] : 0.0;
    }
  } else {      // src[h + r*ld]: 64 consecutive k per wave
    const int h = t & 127, hg = h0 + h;
    const T* a = src + min(hg, k - 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = a[(size_t)min(r0 + 2 * q + (t >> 7), rows - 1) * ld];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 2 * q + (t >> 7), rg = r0 + r;
      tile[r * kRS + (h ^ (r >> 3))] = (rg < rows && hg < k) ? (double)x[q] : 0.0;
    }
  }
  __syncthreads();

  const int r = t >> 3, c = t & 7, rg = r0 + r, sw = r >> 3;
  double v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int el = (e + c) & 15;
    v[el] = tile[r * kRS + ((16 * c + el) ^ sw)];
  }
  int8_t* dst = out + (size_t)rg * k_pad + h0 + 16 * c;

  if (MODE == 0) {
    const int sh = rg < rows ? shift_prime_bits(bits[rg]) : 0;
    int b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double x = fabs(v[e]);
      double cl = ceil(ldexp(x, sh));
      b[e] = x == 0.0 ? 0 : (cl < 1.0 ? 1 : (int)cl);
    }
    uint4 w;
    w.x = pack4(b[0], b[1], b[2], b[3]);
    w.y = pack4(b[4], b[5], b[6], b[7]);
    w.z = pack4(b[8], b[9], b[10], b[11]);
    w.w = pack4(b[12], b[13], b[14], b[15]);
    *reinterpret_cast<uint4*>(dst) = w;
  } else {
    if (rg >= rows) return;   // after the only barrier
    const int sh = shift[rg];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = trunc(ldexp(v[e], sh));
    if (cc.nlimbs == 2) {          // uniform branches
      store_residues_limbs<2>(v, cc, dst, slice);
    } else if (cc.nlimbs == 3) {
      store_residues_limbs<3>(v, cc, dst, slice);
    } else {
      switch (cc.nsteps) {
        case 1: store_residues<1>(v, cc, dst, slice); break;
        case 2: store_residues<2>(v, cc, dst, slice); break;
        case 3: store_residues<3>(v, cc, dst, slice); break;
        default: store_residues<4>(v, cc, dst, slice); break;
      }
    }
  }
}

// Tile order of workgroup b: for the column-major A side (TRANS) row tiles
// vary fastest, so workgroups running together read neighbouring 256-byte
// pieces of the same columns (DRAM pages); for B, whose rows are contiguous
// in k, k tiles vary fastest.
template <bool TRANS>
__device__ inline void slice_tile(int b, int k_pad, int rows_pad, int* kx, int* ry) {
  if (TRANS) {
    const int gy = rows_pad / kTR;
    *kx = b / gy;
    *ry = b % gy;
  } else {
    const int gx = k_pad / kTK;
    *kx = b % gx;
    *ry = b / gx;
  }
}

template <typename T, bool TRANS, int MODE>
__global__ __launch_bounds__(256) void k_slices(const T* __restrict__ src, int ld, int rows, int k,
                                                int k_pad, size_t slice, const uint64_t* __restrict__ bits,
                                                const int* __restrict__ shift, CrtConsts cc,
                                                int8_t* __restrict__ out) {
  int kx, ry;
  slice_tile<TRANS>(blockIdx.x, k_pad, (int)(slice / k_pad), &kx, &ry);
  slices_body<T, TRANS, MODE>(src, ld, rows, k, k_pad, slice, bits, shift, cc, out, kx, ry);
}

// Grouped: A side (TRANS, rows = m) or B side (rows = n) of every problem.
template <typename T, bool ASIDE, int MODE>
__global__ __launch_bounds__(256) void kg_slices(const ProbDesc* __restrict__ P,
                                                 const BlockRef* __restrict__ map,
                                                 const CrtConsts* __restrict__ ctab) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  int kx, ry;
  if (ASIDE) {
    slice_tile<true>(e.y, d.kp, d.mp, &kx, &ry);
    slices_body<T, true, MODE>((const T*)d.A, d.lda, d.m, d.k, d.kp, (size_t)d.mp * d.kp,
                               d.rowbits, d.mu, ctab[d.N], d.As, kx, ry);
  } else {
    slice_tile<false>(e.y, d.kp, d.np, &kx, &ry);
    slices_body<T, false, MODE>((const T*)d.B, d.ldb, d.n, d.k, d.kp, (size_t)d.np * d.kp,
                                d.colbits, d.nu, ctab[d.N], d.Bs, kx, ry);
  }
}

// Planner operands: x = |a| 2^-alpha (alpha = floor(log2 max_h |a_ih|), so
// x < 2) truncated toward zero to BF16 -- every stored value is a lower bound
// of the exact one -- and, per 64-k tile, the FP64 sum of the exact x of each
// row (partial[tile][row], reduced in a fixed order).
template <typename T, bool TRANS>
__global__ __launch_bounds__(256) void k_plan_slices(const T* __restrict__ src, int ld, int rows,
                                                     int k, int k_pad, int rows_pad,
                                                     const uint64_t* __restrict__ bits,
                                                     uint16_t* __restrict__ out,
                                                     double* __restrict__ partial) {
  __shared__ double tile[kPlanTile][kPlanTile + 1];
  const int t = threadIdx.x;
  const int r0 = blockIdx.y * kPlanTile, h0 = blockIdx.x * kPlanTile;
  if (TRANS) {
    const int r = t & 63, rg = r0 + r;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int h = (t >> 6) + 4 * q, hg = h0 + h;
      tile[r][h] = (rg < rows && hg < k) ? (double)src[rg + (size_t)hg * ld] : 0.0;
    }
  } else {
    const int h = t & 63, hg = h0 + h;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = (t >> 6) + 4 * q, rg = r0 + r;
      tile[r][h] = (rg < rows && hg < k) ? (double)src[hg + (size_t)rg * ld] : 0.0;
    }
  }
  __syncthreads();
  const int r = t >> 2, hc = (t & 3) * 16, rg = r0 + r;
  const int sh = rg < rows ? shift_prime_bits(bits[rg]) - 5 : 0;   // -alpha
  uint32_t packed[8];
  double sum = 0.0;
#pragma unroll
  for (int e = 0; e < 16; e += 2) {
    const double x0 = ldexp(fabs(tile[r][hc + e]), sh), x1 = ldexp(fabs(tile[r][hc + e + 1]), sh);
    sum += x0;
    sum += x1;
    const uint32_t b0 = __float_as_uint(__double2float_rz(x0)) >> 16;
    const uint32_t b1 = __float_as_uint(__double2float_rz(x1)) >> 16;
    packed[e >> 1] = b0 | (b1 << 16);
  }
  uint4* dst = reinterpret_cast<uint4*>(out + (size_t)rg * k_pad + h0 + hc);
  dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
  sum += __shfl_xor(sum, 1);
  sum += __shfl_xor(sum, 2);
  if ((t & 3) == 0) partial[(size_t)blockIdx.x * rows_pad + rg] = sum;
}

template <typename T>
void launch_t(hipStream_t s, int mode, bool trans, const T* src, int ld, int rows, int k,
              int rows_pad, int k_pad, const uint64_t* bits, const int* shift, const CrtConsts& cc,
              int8_t* out) {
  dim3 grid((unsigned)((k_pad / kTK) * (rows_pad / kTR)));
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

template <typename T, int MODE>
void group_slices_t(hipStream_t s, bool aside, const ProbDesc* P, const BlockRef* map, int blocks,
                    const CrtConsts* ctab) {
  const dim3 g((unsigned)blocks), b(256);
  if (aside)
    hipLaunchKernelGGL((kg_slices<T, true, MODE>), g, b, 0, s, P, map, ctab);
  else
    hipLaunchKernelGGL((kg_slices<T, false, MODE>), g, b, 0, s, P, map, ctab);
}

}  // namespace

void launch_group_slices(hipStream_t s, Prec pr, int mode, bool aside, const ProbDesc* P,
                         const BlockRef* map, int blocks, const CrtConsts* ctab) {
  if (blocks <= 0) return;
  if (pr == Prec::F64) {
    if (mode == 0)
      group_slices_t<double, 0>(s, aside, P, map, blocks, ctab);
    else
      group_slices_t<double, 1>(s, aside, P, map, blocks, ctab);
  } else {
    if (mode == 0)
      group_slices_t<float, 0>(s, aside, P, map, blocks, ctab);
    else
      group_slices_t<float, 1>(s, aside, P, map, blocks, ctab);
  }
}

void launch_plan_slices(hipStream_t s, Prec pr, bool trans, const void* src, int ld, int rows,
                        int k, int rows_pad, int k_pad, const uint64_t* bits, uint16_t* out,
                        double* partial) {
  dim3 grid(k_pad / kPlanTile, rows_pad / kPlanTile);
  if (pr == Prec::F64) {
    if (trans)
      hipLaunchKernelGGL((k_plan_slices<double, true>), grid, dim3(256), 0, s, (const double*)src,
                         ld, rows, k, k_pad, rows_pad, bits, out, partial);
    else
      hipLaunchKernelGGL((k_plan_slices<double, false>), grid, dim3(256), 0, s, (const double*)src,
                         ld, rows, k, k_pad, rows_pad, bits, out, partial);
  } else {
    if (trans)
      hipLaunchKernelGGL((k_plan_slices<float, true>), grid, dim3(256), 0, s, (const float*)src, ld,
                         rows, k, k_pad, rows_pad, bits, out, partial);
    else
      hipLaunchKernelGGL((k_plan_slices<float, false>), grid, dim3(256), 0, s, (const float*)src, ld,
                         rows, k, k_pad, rows_pad, bits, out, partial);
  }
}

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
