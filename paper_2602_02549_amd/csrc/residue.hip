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
// The LDS rows are 132 doubles apart and the low bits of each column index
// XOR-swizzled, so that the staging stores and the in-order reads
// of a wave spread evenly over 64 four-byte banks, and no thread indexes its
// registers with a per-lane value.
// Each workgroup walks tiles in a grid-stride loop and issues the loads of
// its next tile before computing the current one.
//
// Residues of the scaled integer v = trunc(2^mu a) (|v| < 2^B, B = 6 + floor P')
// are exact in FP64.  v is split once per element into limbs, and per modulus
// r = sum_t v_t c_t with c_0 = 1, c_t = mod(2^(s t), p), |c_t| <= 127, is
// exact and below 2^50; one step r <- r - p * round(r / p) then lands in
// [-(p-1)/2, (p-1)/2] for odd p.
//   two limbs (B <= 90, N = 12..22): v = v_1 2^48 + v_0, |v_0| <= 2^47,
//     |v_1| <= 2^42, so |r| <= 2^47 + 127 * 2^42 < 2^49.4;
//   three limbs (B <= 122, N = 23..31): v = v_2 2^80 + v_1 2^40 + v_0,
//     |v_0|, |v_1| <= 2^39, |v_2| <= 2^42, so |r| <= 128 * 2^39 + 127 * 2^42
//     < 2^49.2.
// Other N take nsteps such steps from v itself (each exact, shrinking |r| by
// ~2^-52 relative; the last starts from |r| < 2^50).  For p = 256 the result
// lies in [-128, 128] and the byte store wraps 128 to -128; 2^48, 2^40 and
// 2^80 are 0 mod 256.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr int kTR = 32;           // slice tile: rows
constexpr int kTK = 128;          // slice tile: k
constexpr int kRS = kTK + 4;      // LDS row stride (doubles)
constexpr int kPlanTile = 64;     // planner operand tile

// Rounding to an integer and reading an integer without the FP64 round and
// convert instructions (which issue at a fraction of the FMA rate): with
// kRound = 1.5 * 2^52, fma(x, y, kRound) is kRound plus the exact product
// x*y rounded to the nearest integer (ties to even) whenever |x*y| < 2^51,
// since doubles in [2^52, 2^53) are the integers; and for an integer-valued
// |x| < 2^31 the low 32 bits of x + kRound are x in two's complement.
constexpr double kRound = 0x1.8p52;

__device__ __forceinline__ double round_prod(double x, double y) {
  return fma(x, y, kRound) - kRound;
}

__device__ __forceinline__ int int_of(double x) { return __double2loint(x + kRound); }

// One exact reduction step r - p * round(r / p) for |r| < 2^50: the rounded
// product is the nearest integer to r / p itself, because |r| |pinv - 1/p|
// <= 2^-3 / p is below the distance 1 / (2p) from r / p to a half-integer
// (odd p), and pinv is exact for p = 256.  The result lies in
// [-(p-1)/2, (p-1)/2] for odd p and in [-128, 128] for p = 256.
__device__ __forceinline__ double reduce_last(double r, double p, double pinv) {
  return fma(-round_prod(r, pinv), p, r);
}

// nsteps reduction steps (the last from |r| < 2^50); NS = 1..4 for N <= 49.
// The earlier steps only shrink |r| exactly, for which rint of the rounded
// product suffices.
template <int NS>
__device__ __forceinline__ int residue_i8(double v, int p, double pinv) {
  double r = v;
#pragma unroll
  for (int s = 0; s + 1 < NS; ++s) {
    const double q = rint(r * pinv);
    r = fma(-q, (double)p, r);
  }
  return int_of(reduce_last(r, (double)p, pinv));
}

// Low bytes of a, b, c, d as one word (byte 0 = a), three byte permutes:
// v_perm_b32 picks bytes 0-3 of its second source with selectors 0-3, of its
// first with 4-7, and zero with 0x0c.
__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d) {
  const uint32_t ab = __builtin_amdgcn_perm((uint32_t)b, (uint32_t)a, 0x0c0c0400u);
  const uint32_t cd = __builtin_amdgcn_perm((uint32_t)d, (uint32_t)c, 0x0c0c0400u);
  return __builtin_amdgcn_perm(cd, ab, 0x05040100u);
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

// Limb form of the residues: L = 2 limbs split at 2^48, or L = 3 limbs
// split at 2^80 and 2^40 (bounds in the file header).
template <int L>
__device__ __forceinline__ void store_residues_limbs(const double (&v)[16], const CrtConsts& cc,
                                                     int8_t* __restrict__ dst, size_t slice) {
  static_assert(L == 2 || L == 3, "limbs");
  constexpr double kS = L == 2 ? 0x1p48 : 0x1p40, kSinv = L == 2 ? 0x1p-48 : 0x1p-40;
  double lo[16], mid[16], hi[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    double rem = v[e];
    if (L == 3) {
      hi[e] = round_prod(rem, 0x1p-80);        // |v| < 2^122: |hi| <= 2^42
      rem = fma(-hi[e], 0x1p80, rem);          // exact, |rem| <= 2^79
    }
    mid[e] = round_prod(rem, kSinv);
    lo[e] = fma(-mid[e], kS, rem);             // exact, |lo| <= 2^47 (L = 2), 2^39 (L = 3)
  }
  for (int l = 0; l < cc.N; ++l) {
    const double p = (double)cc.p[l];
    const double pinv = cc.pinv[l];
    const double c1 = reduce_last(kS, p, pinv);                     // mod(2^s, p)
    const double c2 = L == 3 ? reduce_last(c1 * c1, p, pinv) : 0.0;  // mod(2^80, p)
    int b[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double r = fma(mid[e], c1, lo[e]);
      if (L == 3) r = fma(hi[e], c2, r);
      b[e] = int_of(reduce_last(r, p, pinv));
    }
    uint4 w;
    w.x = pack4(b[0], b[1], b[2], b[3]);
    w.y = pack4(b[4], b[5], b[6], b[7]);
    w.z = pack4(b[8], b[9], b[10], b[11]);
    w.w = pack4(b[12], b[13], b[14], b[15]);
    *reinterpret_cast<uint4*>(dst + (size_t)l * slice) = w;
  }
}

// Workgroup barrier for the LDS tile only: it waits for this wave's LDS
// (and scalar) traffic, not for its global loads, so the next tile's loads
// stay in flight across it.  The memory clobber keeps the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The 16 source elements of one thread for the tile at rows r0.., k h0..;
// all 16 loads go out before any is used.  Addresses are clamped into the
// matrix (rows, k >= 1); out-of-range elements are zeroed when staged.
template <typename T, bool TRANS>
__device__ __forceinline__ void tile_loads(const T* __restrict__ src, int ld, int rows, int k,
                                           int r0, int h0, T (&x)[16]) {
  const int t = threadIdx.x;
  if (TRANS) {  // src[r + h*ld]: 32 consecutive rows per half-wave, two columns per wave
    const T* a = src + min(r0 + (t & 31), rows - 1);
    const int hb = h0 + (t >> 5);
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = a[(size_t)min(hb + 8 * q, k - 1) * ld];
  } else {      // src[h + r*ld]: 128 consecutive k per half-block
    const T* a = src + min(h0 + (t & 127), k - 1);
    const int rb = r0 + (t >> 7);
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = a[(size_t)min(rb + 2 * q, rows - 1) * ld];
  }
}

// Per-row input of the thread's output row r0 + t/8 (clamped): the abs-max
// bit pattern (mode 0) or the shift mu / nu (mode 1).
template <int MODE>
__device__ __forceinline__ int64_t row_aux(const void* __restrict__ aux, int rows, int r0) {
  const int rg = min(r0 + (int)(threadIdx.x >> 3), rows - 1);
  if (MODE != 1) return (int64_t)static_cast<const uint64_t*>(aux)[rg];
  return static_cast<const int*>(aux)[rg];
}

// LDS position of element (r, h) of a tile:
//   r * kRS + (h ^ (((h / 32) ^ (r / 8)) & 3)),
// rows kRS doubles apart and the low two bits of h XORed with bits of h / 32
// and r / 8.  Counted over 64 four-byte banks, both staging patterns and the
// in-order reads of tile_finish put exactly two of a wave's 8-byte accesses
// on each bank.  tile_stage and tile_finish address it as four base
// addresses plus constant offsets (the XOR term is constant within each
// group of four steps).

// Writes the thread's 16 elements into the LDS tile (zero outside the matrix).
// Within each group of four steps q the XOR term of the position map is constant
// (h / 32 and r / 8 depend on q / 4 only), so the positions are four bases
// plus constant offsets.
template <typename T, bool TRANS>
__device__ __forceinline__ void tile_stage(const T (&x)[16], int rows, int k, int r0, int h0,
                                           double* tile) {
  const int t = threadIdx.x;
  if (TRANS) {  // element (r, h = hb + 8q): position r*kRS + 8q + (hb ^ ((q/4 ^ r/8) & 3))
    const int r = t & 31, rg = r0 + r, hb = t >> 5;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double* base = tile + r * kRS + (hb ^ ((j ^ (r >> 3)) & 3));
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 4 * j + i, h = hb + 8 * q;
        base[8 * q] = (rg < rows && h0 + h < k) ? (double)x[q] : 0.0;
      }
    }
  } else {      // element (r = 2q + t/128, h): position r*kRS + (h ^ ((h/32 ^ q/4) & 3))
    const int h = t & 127, hg = h0 + h, rb = t >> 7;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double* base = tile + rb * kRS + (h ^ (((h >> 5) ^ j) & 3));
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 4 * j + i, rg = r0 + 2 * q + rb;
        base[2 * q * kRS] = (rg < rows && hg < k) ? (double)x[q] : 0.0;
      }
    }
  }
}

// Each thread reads 16 consecutive k of one row from the staged tile and
// writes 16 bytes per slice (mode 0: Abar; mode 1: the N residues).
// Residue paths of mode 1: limbs (2 or 3) or exact reduction steps (1, 3 or
// 4; the limbs cover every N that would take two steps, and an extra step is
// exact anyway); kAnyPath chooses at run time from the constants (grouped
// launches, whose problems differ in N).
enum ResiduePath { kLimbs2, kLimbs3, kSteps1, kSteps3, kSteps4, kAnyPath };

int residue_path(const CrtConsts& cc) {
  if (cc.nlimbs == 2) return kLimbs2;
  if (cc.nlimbs == 3) return kLimbs3;
  return cc.nsteps <= 1 ? kSteps1 : cc.nsteps <= 3 ? kSteps3 : kSteps4;
}

template <int PATH>
__device__ __forceinline__ void store_residues_path(const double (&v)[16], const CrtConsts& cc,
                                                    int8_t* __restrict__ dst, size_t slice) {
  switch (PATH) {
    case kLimbs2: store_residues_limbs<2>(v, cc, dst, slice); break;
    case kLimbs3: store_residues_limbs<3>(v, cc, dst, slice); break;
    case kSteps1: store_residues<1>(v, cc, dst, slice); break;
    case kSteps3: store_residues<3>(v, cc, dst, slice); break;
    case kSteps4: store_residues<4>(v, cc, dst, slice); break;
    default:
      if (cc.nlimbs == 2) {          // uniform branches
        store_residues_limbs<2>(v, cc, dst, slice);
      } else if (cc.nlimbs == 3) {
        store_residues_limbs<3>(v, cc, dst, slice);
      } else if (cc.nsteps <= 1) {
        store_residues<1>(v, cc, dst, slice);
      } else if (cc.nsteps <= 3) {
        store_residues<3>(v, cc, dst, slice);
      } else {
        store_residues<4>(v, cc, dst, slice);
      }
  }
}

template <int MODE, int PATH>
__device__ __forceinline__ void tile_finish(const double* tile, int64_t aux, int rows, int k_pad,
                                            size_t slice, const CrtConsts& cc,
                                            int8_t* __restrict__ out, int r0, int h0) {
  const int t = threadIdx.x;
  const int r = t >> 3, c = t & 7, rg = r0 + r;
  // element (r, 16c + e): position r*kRS + 16c + 4(e/4) + ((e%4) ^ g)
  const int g = ((c >> 1) ^ (r >> 3)) & 3;
  double v[16];
#pragma unroll
  for (int el = 0; el < 4; ++el) {
    const double* base = tile + r * kRS + 16 * c + (el ^ g);
#pragma unroll
    for (int eh = 0; eh < 4; ++eh) v[4 * eh + el] = base[4 * eh];
  }
  int8_t* dst = out + (size_t)rg * k_pad + h0 + 16 * c;

  if (MODE != 1) {
    const int sh = rg < rows ? shift_prime_bits((uint64_t)aux) - (MODE == 2 ? 1 : 0) : 0;
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
  } else if (rg < rows) {
    const int sh = (int)aux;
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = trunc(ldexp(v[e], sh));
    store_residues_path<PATH>(v, cc, dst, slice);
  }
}

// Tile b of an operand with gy row tiles of 32: for the column-major A side
// (TRANS) row tiles vary fastest, so workgroups running together read
// neighbouring 256-byte pieces of the same columns (DRAM pages); for B, whose
// rows are contiguous in k, k tiles vary fastest.
template <bool TRANS>
__device__ inline void slice_tile(int b, int k_pad, int gy, int* kx, int* ry) {
  if (TRANS) {
    *kx = b / gy;
    *ry = b % gy;
  } else {
    const int gx = k_pad / kTK;
    *kx = b % gx;
    *ry = b / gx;
  }
}

// Grid-stride loop over `tiles` tiles (row tiles: gy; mode 1 leaves out the
// tiles of padding rows, whose residues no product of real rows reads; Abar
// and Bbar padding must stay zero, since the scaling product's maxima cover
// whole rows and columns).  Each workgroup stages tile i in LDS, issues the
// loads of its next tile, and only then computes and stores tile i, so that
// HBM reads overlap the residue arithmetic.
template <typename T, bool TRANS, int MODE, int PATH>
__global__ __launch_bounds__(256) void k_slices(const T* __restrict__ src, int ld, int rows, int k,
                                                int k_pad, int gy, int tiles, size_t slice,
                                                const void* __restrict__ aux, CrtConsts cc,
                                                int8_t* __restrict__ out) {
  __shared__ double tile[kTR * kRS];
  int i = blockIdx.x;
  if (i >= tiles) return;
  int kx, ry;
  slice_tile<TRANS>(i, k_pad, gy, &kx, &ry);
  T x[16];
  tile_loads<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x);
  int64_t xa = row_aux<MODE>(aux, rows, ry * kTR);
  for (;;) {
    const int r0 = ry * kTR, h0 = kx * kTK;
    lds_barrier();                 // every wave is done with the previous tile
    tile_stage<T, TRANS>(x, rows, k, r0, h0, tile);
    __asm__ volatile("" ::: "memory");  // x is free: the next loads reuse its registers
    const int64_t a = xa;
    const int ni = i + (int)gridDim.x;
    if (ni < tiles) {
      slice_tile<TRANS>(ni, k_pad, gy, &kx, &ry);
      tile_loads<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x);
      xa = row_aux<MODE>(aux, rows, ry * kTR);
    }
    lds_barrier();                 // the tile is staged
    tile_finish<MODE, PATH>(tile, a, rows, k_pad, slice, cc, out, r0, h0);
    if (ni >= tiles) break;
    i = ni;
  }
}

// ---- complex operands of the 3-product form (ozaki2_zgemm3m) -------------
// The source holds interleaved (re, im) pairs, column-major, ld in complex
// elements.  Both parts of a tile are loaded together (the complex matrix is
// read once per pass) and staged one after the other through the one LDS
// tile of k_slices, each thread taking its 16 values of each part into
// registers:
//   mode 2: Abar of the complex rows, ceil(2^(mu'-1) |re|) + ceil(2^(mu'-1) |im|)
//     (each at most 32), one slice at out;
//   mode 1: the residues of A'r, A'i and A'r + A'i, N slices each, at out,
//     out + N slice and out + 2 N slice.  Per modulus the residues of the two
//     parts come from the residue path's arithmetic, and the third is their
//     sum brought back into the symmetric range by one correction.

// Residue of one value for modulus (p, pd, pinv) on the residue path; the
// limb paths split the value again for each modulus, which keeps no
// per-value state across moduli (registers stay free for the next tile's
// loads).  c1 = mod(2^s, p) and c2 = mod(2^80, p) of the limb paths.
template <int PATH>
__device__ __forceinline__ int residue_one(double v, int p, double pd, double pinv, double c1,
                                           double c2) {
  if constexpr (PATH == kLimbs2) {
    const double mid = round_prod(v, 0x1p-48);
    const double lo = fma(-mid, 0x1p48, v);            // exact, |lo| <= 2^47
    return int_of(reduce_last(fma(mid, c1, lo), pd, pinv));
  } else if constexpr (PATH == kLimbs3) {
    const double hi = round_prod(v, 0x1p-80);
    const double rem = fma(-hi, 0x1p80, v);            // exact, |rem| <= 2^79
    const double mid = round_prod(rem, 0x1p-40);
    const double lo = fma(-mid, 0x1p40, rem);          // exact, |lo| <= 2^39
    return int_of(reduce_last(fma(hi, c2, fma(mid, c1, lo)), pd, pinv));
  } else {
    return residue_i8<PATH == kSteps1 ? 1 : PATH == kSteps3 ? 3 : 4>(v, p, pinv);
  }
}

// The thread's 16 staged elements of its row (the order of tile_finish).
__device__ __forceinline__ void tile_row16(const double* tile, double (&v)[16]) {
  const int t = threadIdx.x;
  const int r = t >> 3, c = t & 7;
  const int g = ((c >> 1) ^ (r >> 3)) & 3;
#pragma unroll
  for (int el = 0; el < 4; ++el) {
    const double* base = tile + r * kRS + 16 * c + (el ^ g);
#pragma unroll
    for (int eh = 0; eh < 4; ++eh) v[4 * eh + el] = base[4 * eh];
  }
}

template <int MODE, int PATH>
__device__ __forceinline__ void tile_finish_cx(double (&vr)[16], double (&vi)[16], int64_t aux,
                                               int rows, int k_pad, size_t slice,
                                               const CrtConsts& cc, int8_t* __restrict__ out,
                                               int r0, int h0) {
  const int t = threadIdx.x;
  const int rg = r0 + (t >> 3);
  int8_t* dst = out + (size_t)rg * k_pad + h0 + 16 * (t & 7);
  if constexpr (MODE == 2) {
    const int sh = rg < rows ? shift_prime_bits((uint64_t)aux) - 1 : 0;
    auto bar = [&](double v) {
      const double x = fabs(v);
      const double cl = ceil(ldexp(x, sh));
      return x == 0.0 ? 0 : (cl < 1.0 ? 1 : (int)cl);
    };
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = pack4(bar(vr[4 * q]) + bar(vi[4 * q]), bar(vr[4 * q + 1]) + bar(vi[4 * q + 1]),
                   bar(vr[4 * q + 2]) + bar(vi[4 * q + 2]), bar(vr[4 * q + 3]) + bar(vi[4 * q + 3]));
    *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
  } else {
    if (rg >= rows) return;
    const int sh = (int)aux;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      vr[e] = trunc(ldexp(vr[e], sh));
      vi[e] = trunc(ldexp(vi[e], sh));
    }
    const size_t set = (size_t)cc.N * slice;
    for (int l = 0; l < cc.N; ++l) {
      const int p = cc.p[l], hi = (p - 1) / 2, lo = hi + 1 - p;
      const double pd = (double)p, pinv = cc.pinv[l];
      double c1 = 0.0, c2 = 0.0;
      if constexpr (PATH == kLimbs2) c1 = reduce_last(0x1p48, pd, pinv);
      if constexpr (PATH == kLimbs3) {
        c1 = reduce_last(0x1p40, pd, pinv);
        c2 = reduce_last(c1 * c1, pd, pinv);
      }
      // residues of the parts in [-(p-1)/2, (p-1)/2] (odd p) or [-128, 128]
      // (p = 256, stored as bytes mod 256): one correction puts their sum in
      // the range
      uint32_t wr[4], wi[4], ws[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int br[4], bi[4], bs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          br[u] = residue_one<PATH>(vr[4 * q + u], p, pd, pinv, c1, c2);
          bi[u] = residue_one<PATH>(vi[4 * q + u], p, pd, pinv, c1, c2);
          int x = br[u] + bi[u];
          x -= x > hi ? p : 0;
          bs[u] = x + (x < lo ? p : 0);
        }
        wr[q] = pack4(br[0], br[1], br[2], br[3]);
        wi[q] = pack4(bi[0], bi[1], bi[2], bi[3]);
        ws[q] = pack4(bs[0], bs[1], bs[2], bs[3]);
      }
      int8_t* d = dst + (size_t)l * slice;
      *reinterpret_cast<uint4*>(d) = make_uint4(wr[0], wr[1], wr[2], wr[3]);
      *reinterpret_cast<uint4*>(d + set) = make_uint4(wi[0], wi[1], wi[2], wi[3]);
      *reinterpret_cast<uint4*>(d + 2 * set) = make_uint4(ws[0], ws[1], ws[2], ws[3]);
    }
  }
}

template <typename T, bool TRANS>
__device__ __forceinline__ void tile_loads_cx(const T* __restrict__ src, int ld, int rows, int k,
                                              int r0, int h0, T (&x)[16], T (&y)[16]) {
  const int t = threadIdx.x;
  if (TRANS) {  // element (r, h) at src[2 (r + h ld)]: as tile_loads, pairs
    const T* a = src + 2 * (size_t)min(r0 + (t & 31), rows - 1);
    const int hb = h0 + (t >> 5);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const T* e = a + 2 * ((size_t)min(hb + 8 * q, k - 1) * ld);
      x[q] = e[0];
      y[q] = e[1];
    }
  } else {      // element (h, r) at src[2 (h + r ld)]
    const T* a = src + 2 * (size_t)min(h0 + (t & 127), k - 1);
    const int rb = r0 + (t >> 7);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const T* e = a + 2 * ((size_t)min(rb + 2 * q, rows - 1) * ld);
      x[q] = e[0];
      y[q] = e[1];
    }
  }
}

// The grid-stride loop of k_slices over complex tiles: the real parts are
// staged and read back, then the imaginary parts, then the next tile's loads
// go out before the arithmetic of this one.
template <typename T, bool TRANS, int MODE, int PATH>
__global__ __launch_bounds__(256) void k_slices_cx(const T* __restrict__ src, int ld, int rows,
                                                   int k, int k_pad, int gy, int tiles,
                                                   size_t slice, const void* __restrict__ aux,
                                                   CrtConsts cc, int8_t* __restrict__ out) {
  __shared__ double tile[kTR * kRS];
  int i = blockIdx.x;
  if (i >= tiles) return;
  int kx, ry;
  slice_tile<TRANS>(i, k_pad, gy, &kx, &ry);
  T x[16], y[16];
  tile_loads_cx<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x, y);
  int64_t xa = row_aux<MODE>(aux, rows, ry * kTR);
  for (;;) {
    const int r0 = ry * kTR, h0 = kx * kTK;
    double vr[16], vi[16];
    lds_barrier();                 // every wave is done with the previous tile
    tile_stage<T, TRANS>(x, rows, k, r0, h0, tile);
    lds_barrier();
    tile_row16(tile, vr);
    lds_barrier();
    tile_stage<T, TRANS>(y, rows, k, r0, h0, tile);
    __asm__ volatile("" ::: "memory");  // x, y are free: the next loads reuse their registers
    const int64_t a = xa;
    const int ni = i + (int)gridDim.x;
    if (ni < tiles) {
      slice_tile<TRANS>(ni, k_pad, gy, &kx, &ry);
      tile_loads_cx<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x, y);
      xa = row_aux<MODE>(aux, rows, ry * kTR);
    }
    lds_barrier();
    tile_row16(tile, vi);
    tile_finish_cx<MODE, PATH>(vr, vi, a, rows, k_pad, slice, cc, out, r0, h0);
    if (ni >= tiles) break;
    i = ni;
  }
}

// ---- the real embedding of a complex product (ozaki2_zgemm) --------------
// Ahat = [[Ar, -Ai], [Ai, Ar]] and Bhat = [[Br], [Bi]] written as slices
// straight from the interleaved complex source: k-half kh (slice rows 2 kh
// long), and on the A side row half `half`.  A complex element (i, h) of A
// lands in Ahat at (i, h) as re, (i, kh + h) as -im, (half + i, h) as im and
// (half + i, kh + h) as re; of B at row j of Bhat^T: (j, h) re, (j, kh + h) im.
//   mode 0: the bars; rows i and half + i share mu'_i (the same maximum).
//   mode 1: the residues; row i is scaled by shift[i], row half + i by
//     shift[half + i] (their Cbar maxima differ).  The residue of -x is the
//     negated residue of x (the reduction is odd-symmetric; for p = 256 the
//     byte of -(-128) wraps to -128 as the real kernel's 128 does).
template <int MODE, int PATH, bool ASIDE>
__device__ __forceinline__ void tile_finish_emb(const double (&vr)[16], const double (&vi)[16],
                                                const void* __restrict__ aux, int rows, int ldo,
                                                int kh, int half, size_t slice,
                                                const CrtConsts& cc, int8_t* __restrict__ out,
                                                int r0, int h0) {
  const int t = threadIdx.x;
  const int rg = r0 + (t >> 3);
  int8_t* d0 = out + (size_t)rg * ldo + h0 + 16 * (t & 7);    // (rg, h)
  int8_t* d1 = d0 + kh;                                         // (rg, kh + h)
  const size_t dh = (size_t)half * ldo;                         // to row half + rg
  if constexpr (MODE == 0) {
    const int sh = rg < rows
                       ? shift_prime_bits(static_cast<const uint64_t*>(aux)[min(rg, rows - 1)])
                       : 0;
    auto bar = [&](double v) {
      const double x = fabs(v);
      const double cl = ceil(ldexp(x, sh));
      return x == 0.0 ? 0 : (cl < 1.0 ? 1 : (int)cl);
    };
    uint32_t wr[4], wi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wr[q] = pack4(bar(vr[4 * q]), bar(vr[4 * q + 1]), bar(vr[4 * q + 2]), bar(vr[4 * q + 3]));
      wi[q] = pack4(bar(vi[4 * q]), bar(vi[4 * q + 1]), bar(vi[4 * q + 2]), bar(vi[4 * q + 3]));
    }
    const uint4 ur = make_uint4(wr[0], wr[1], wr[2], wr[3]), ui = make_uint4(wi[0], wi[1], wi[2], wi[3]);
    *reinterpret_cast<uint4*>(d0) = ur;
    *reinterpret_cast<uint4*>(d1) = ui;
    if (ASIDE) {
      *reinterpret_cast<uint4*>(d0 + dh) = ui;
      *reinterpret_cast<uint4*>(d1 + dh) = ur;
    }
  } else {
    if (rg >= rows) return;
    const int* sh = static_cast<const int*>(aux);
    // block 0: rows rg (A side) or the only row (B side); block 1: row half + rg
    for (int blk = 0; blk < (ASIDE ? 2 : 1); ++blk) {
      const int e2 = sh[rg + blk * half];
      double xr[16], xi[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        xr[e] = trunc(ldexp(vr[e], e2));
        xi[e] = trunc(ldexp(vi[e], e2));
      }
      int8_t* b0 = d0 + blk * dh;
      int8_t* b1 = d1 + blk * dh;
      for (int l = 0; l < cc.N; ++l) {
        const int p = cc.p[l];
        const double pd = (double)p, pinv = cc.pinv[l];
        double c1 = 0.0, c2 = 0.0;
        if constexpr (PATH == kLimbs2) c1 = reduce_last(0x1p48, pd, pinv);
        if constexpr (PATH == kLimbs3) {
          c1 = reduce_last(0x1p40, pd, pinv);
          c2 = reduce_last(c1 * c1, pd, pinv);
        }
        uint32_t first[4], second[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int br[4], bi[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            br[u] = residue_one<PATH>(xr[4 * q + u], p, pd, pinv, c1, c2);
            bi[u] = residue_one<PATH>(xi[4 * q + u], p, pd, pinv, c1, c2);
          }
          // A side: row rg holds [re, -im], row half + rg [im, re]; B side [re, im]
          if (!ASIDE) {
            first[q] = pack4(br[0], br[1], br[2], br[3]);
            second[q] = pack4(bi[0], bi[1], bi[2], bi[3]);
          } else if (blk == 0) {
            first[q] = pack4(br[0], br[1], br[2], br[3]);
            second[q] = pack4(-bi[0], -bi[1], -bi[2], -bi[3]);
          } else {
            first[q] = pack4(bi[0], bi[1], bi[2], bi[3]);
            second[q] = pack4(br[0], br[1], br[2], br[3]);
          }
        }
        *reinterpret_cast<uint4*>(b0 + (size_t)l * slice) =
            make_uint4(first[0], first[1], first[2], first[3]);
        *reinterpret_cast<uint4*>(b1 + (size_t)l * slice) =
            make_uint4(second[0], second[1], second[2], second[3]);
      }
    }
  }
}

// Grid-stride loop as k_slices_cx over the complex source's tiles (kh / 128
// k tiles by gy row tiles).
template <typename T, bool TRANS, int MODE, int PATH>
__global__ __launch_bounds__(256) void k_slices_emb(const T* __restrict__ src, int ld, int rows,
                                                    int k, int kh, int gy, int tiles, int half,
                                                    size_t slice, const void* __restrict__ aux,
                                                    CrtConsts cc, int8_t* __restrict__ out) {
  // The A side's residues (two row blocks, four stores per modulus) hold
  // the most registers: there the next tile's loads are not issued early,
  // which lets two workgroups share a CU instead of one.
  constexpr bool kPrefetch = !(TRANS && MODE == 1);
  __shared__ double tile[kTR * kRS];
  int i = blockIdx.x;
  if (i >= tiles) return;
  int kx, ry;
  slice_tile<TRANS>(i, kh, gy, &kx, &ry);
  T x[16], y[16];
  if (kPrefetch) tile_loads_cx<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x, y);
  for (;;) {
    const int r0 = ry * kTR, h0 = kx * kTK;
    double vr[16], vi[16];
    if (!kPrefetch) tile_loads_cx<T, TRANS>(src, ld, rows, k, r0, h0, x, y);
    lds_barrier();                 // every wave is done with the previous tile
    tile_stage<T, TRANS>(x, rows, k, r0, h0, tile);
    lds_barrier();
    tile_row16(tile, vr);
    lds_barrier();
    tile_stage<T, TRANS>(y, rows, k, r0, h0, tile);
    __asm__ volatile("" ::: "memory");  // x, y are free: the next loads reuse their registers
    const int ni = i + (int)gridDim.x;
    if (ni < tiles) {
      slice_tile<TRANS>(ni, kh, gy, &kx, &ry);
      if (kPrefetch) tile_loads_cx<T, TRANS>(src, ld, rows, k, ry * kTR, kx * kTK, x, y);
    }
    lds_barrier();
    tile_row16(tile, vi);
    tile_finish_emb<MODE, PATH, TRANS>(vr, vi, aux, rows, 2 * kh, kh, half, slice, cc, out, r0,
                                       h0);
    if (ni >= tiles) break;
    i = ni;
  }
}

// One tile of the grouped launch: which problem side and where.
struct TileJob {
  const void* src;
  const void* aux;
  int8_t* out;
  size_t slice;
  int ld, rows, k, k_pad, r0, h0, N;
};

// Map entry i of the grouped launch; false for a mode-1 tile of padding rows.
template <bool ASIDE, int MODE>
__device__ __forceinline__ bool tile_job(const ProbDesc* __restrict__ P,
                                         const BlockRef* __restrict__ map, int i, TileJob* j) {
  const BlockRef e = map[i];
  const ProbDesc& d = P[e.x];
  const int rows = ASIDE ? d.m : d.n, rows_pad = ASIDE ? d.mp : d.np;
  int kx, ry;
  slice_tile<ASIDE>(e.y, d.kp, rows_pad / kTR, &kx, &ry);
  j->r0 = ry * kTR;
  j->h0 = kx * kTK;
  if (MODE == 1 && j->r0 >= rows) return false;
  j->src = ASIDE ? d.A : d.B;
  j->aux = MODE == 0 ? (const void*)(ASIDE ? d.rowbits : d.colbits)
                     : (const void*)(ASIDE ? d.mu : d.nu);
  j->out = ASIDE ? d.As : d.Bs;
  j->slice = (size_t)rows_pad * d.kp;
  j->ld = ASIDE ? d.lda : d.ldb;
  j->rows = rows;
  j->k = d.k;
  j->k_pad = d.kp;
  j->N = d.N;
  return true;
}

// Grouped: A side (TRANS, rows = m) or B side (rows = n) of every problem;
// the same grid-stride loop over the `tiles` entries of the block map.
template <typename T, bool ASIDE, int MODE, int PATH>
__global__ __launch_bounds__(256) void kg_slices(const ProbDesc* __restrict__ P,
                                                 const BlockRef* __restrict__ map, int tiles,
                                                 const CrtConsts* __restrict__ ctab) {
  __shared__ double tile[kTR * kRS];
  const int G = (int)gridDim.x;
  int i = blockIdx.x;
  TileJob cur;
  while (i < tiles && !tile_job<ASIDE, MODE>(P, map, i, &cur)) i += G;
  if (i >= tiles) return;
  T x[16];
  tile_loads<T, ASIDE>(static_cast<const T*>(cur.src), cur.ld, cur.rows, cur.k, cur.r0, cur.h0, x);
  int64_t xa = row_aux<MODE>(cur.aux, cur.rows, cur.r0);
  for (;;) {
    lds_barrier();
    tile_stage<T, ASIDE>(x, cur.rows, cur.k, cur.r0, cur.h0, tile);
    __asm__ volatile("" ::: "memory");
    const int64_t a = xa;
    TileJob nxt;
    int ni = i + G;
    while (ni < tiles && !tile_job<ASIDE, MODE>(P, map, ni, &nxt)) ni += G;
    if (ni < tiles) {
      tile_loads<T, ASIDE>(static_cast<const T*>(nxt.src), nxt.ld, nxt.rows, nxt.k, nxt.r0,
                           nxt.h0, x);
      xa = row_aux<MODE>(nxt.aux, nxt.rows, nxt.r0);
    }
    lds_barrier();
    tile_finish<MODE, PATH>(tile, a, cur.rows, cur.k_pad, cur.slice, ctab[cur.N], cur.out, cur.r0,
                            cur.h0);
    if (ni >= tiles) break;
    i = ni;
    cur = nxt;
  }
}

// Planner operands: x = |a| 2^-alpha (alpha = floor(log2 max_h |a_ih|), so
// x < 2) truncated toward zero to BF16 -- every stored value is a lower bound
// of the exact one -- and, per 64-k tile, the FP64 sum of the exact x of each
// row (partial[tile][row], reduced in a fixed order).  Workgroups walk the
// 64 x 64 tiles in a grid-stride loop and load the next tile into registers
// before they convert the current one.
template <typename T, bool TRANS>
__global__ __launch_bounds__(256) void k_plan_slices(const T* __restrict__ src, int ld, int rows,
                                                     int k, int k_pad, int rows_pad,
                                                     const uint64_t* __restrict__ bits,
                                                     uint16_t* __restrict__ out,
                                                     double* __restrict__ partial) {
  __shared__ double tile[kPlanTile][kPlanTile + 1];
  const int t = threadIdx.x;
  const int tk = k_pad / kPlanTile;
  const int ntiles = tk * (rows_pad / kPlanTile);
  int id = blockIdx.x;
  if (id >= ntiles) return;   // whole workgroup, before any barrier
  // thread t stages element (r, h) = (t & 63, (t >> 6) + 4q) of the tile
  // (TRANS: rows contiguous in memory) or (r, h) = ((t >> 6) + 4q, t & 63)
  auto load = [&](int tid, T (&x)[16]) {
    const int r0 = (tid / tk) * kPlanTile, h0 = (tid % tk) * kPlanTile;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int a = t & 63, b = (t >> 6) + 4 * q;
      const int rg = r0 + (TRANS ? a : b), hg = h0 + (TRANS ? b : a);
      x[q] = (rg < rows && hg < k) ? (TRANS ? src[rg + (size_t)hg * ld] : src[hg + (size_t)rg * ld])
                                   : (T)0;
    }
  };
  T x[16];
  load(id, x);
  for (;;) {
    __syncthreads();   // the previous tile has been read
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int a = t & 63, b = (t >> 6) + 4 * q;
      if (TRANS)
        tile[a][b] = (double)x[q];
      else
        tile[b][a] = (double)x[q];
    }
    __syncthreads();
    const int cur = id;
    id += (int)gridDim.x;
    if (id < ntiles) load(id, x);
    const int r0 = (cur / tk) * kPlanTile, h0 = (cur % tk) * kPlanTile;
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
    if ((t & 3) == 0) partial[(size_t)(cur % tk) * rows_pad + rg] = sum;
    if (id >= ntiles) break;
  }
}

// Resident workgroups per compute unit of each slice kernel and compute
// units per device, filled once per device by init_slice_launch (outside
// any stream capture); a grid-stride launch uses at most that many
// workgroups.  Index: [float][trans / A side][variant], variant 0 = mode 0,
// 1 + path = mode 1 on that residue path (kAnyPath: chosen per tile), and
// the same plus kGrouped for the grouped kernels.
constexpr int kMaxDevices = 64;
constexpr int kGrouped = 2 + kAnyPath;
constexpr int kVariants = 2 * kGrouped;
std::atomic<int> g_cus[kMaxDevices];
std::atomic<int> g_occ[2][2][kVariants];
std::atomic<int> g_occ_cx[2][2][kGrouped];   // k_slices_cx: variant 0 = mode 2, 1 + path
std::atomic<int> g_occ_emb[2][2][kGrouped];  // k_slices_emb: variant 0 = mode 0, 1 + path

template <typename K>
int resident_per_cu(K* kern) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kern), 256, 0) !=
          hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

template <typename T, bool TR>
void fill_occ() {
  std::atomic<int>* o = g_occ[std::is_same<T, float>::value ? 1 : 0][TR ? 1 : 0];
  o[0] = resident_per_cu(k_slices<T, TR, 0, kAnyPath>);
  o[1 + kLimbs2] = resident_per_cu(k_slices<T, TR, 1, kLimbs2>);
  o[1 + kLimbs3] = resident_per_cu(k_slices<T, TR, 1, kLimbs3>);
  o[1 + kSteps1] = resident_per_cu(k_slices<T, TR, 1, kSteps1>);
  o[1 + kSteps3] = resident_per_cu(k_slices<T, TR, 1, kSteps3>);
  o[1 + kSteps4] = resident_per_cu(k_slices<T, TR, 1, kSteps4>);
  o[kGrouped] = resident_per_cu(kg_slices<T, TR, 0, kAnyPath>);
  o[kGrouped + 1 + kLimbs2] = resident_per_cu(kg_slices<T, TR, 1, kLimbs2>);
  o[kGrouped + 1 + kLimbs3] = resident_per_cu(kg_slices<T, TR, 1, kLimbs3>);
  o[kGrouped + 1 + kSteps1] = resident_per_cu(kg_slices<T, TR, 1, kSteps1>);
  o[kGrouped + 1 + kSteps3] = resident_per_cu(kg_slices<T, TR, 1, kSteps3>);
  o[kGrouped + 1 + kSteps4] = resident_per_cu(kg_slices<T, TR, 1, kSteps4>);
  o[kGrouped + 1 + kAnyPath] = resident_per_cu(kg_slices<T, TR, 1, kAnyPath>);
  std::atomic<int>* c = g_occ_cx[std::is_same<T, float>::value ? 1 : 0][TR ? 1 : 0];
  c[0] = resident_per_cu(k_slices_cx<T, TR, 2, kAnyPath>);
  c[1 + kLimbs2] = resident_per_cu(k_slices_cx<T, TR, 1, kLimbs2>);
  c[1 + kLimbs3] = resident_per_cu(k_slices_cx<T, TR, 1, kLimbs3>);
  c[1 + kSteps1] = resident_per_cu(k_slices_cx<T, TR, 1, kSteps1>);
  c[1 + kSteps3] = resident_per_cu(k_slices_cx<T, TR, 1, kSteps3>);
  c[1 + kSteps4] = resident_per_cu(k_slices_cx<T, TR, 1, kSteps4>);
  std::atomic<int>* b = g_occ_emb[std::is_same<T, float>::value ? 1 : 0][TR ? 1 : 0];
  b[0] = resident_per_cu(k_slices_emb<T, TR, 0, kAnyPath>);
  b[1 + kLimbs2] = resident_per_cu(k_slices_emb<T, TR, 1, kLimbs2>);
  b[1 + kLimbs3] = resident_per_cu(k_slices_emb<T, TR, 1, kLimbs3>);
  b[1 + kSteps1] = resident_per_cu(k_slices_emb<T, TR, 1, kSteps1>);
  b[1 + kSteps3] = resident_per_cu(k_slices_emb<T, TR, 1, kSteps3>);
  b[1 + kSteps4] = resident_per_cu(k_slices_emb<T, TR, 1, kSteps4>);
}

// Workgroups for `tiles` tiles: all resident slots of the device, or one per
// tile if the device's figures are unknown.  A positive g_slice_cap (a test
// knob set through ozaki2_debug_tuning) caps the count, so that each
// workgroup walks many tiles.
// kind: 0 = k_slices, 1 = k_slices_cx, 2 = k_slices_emb.
int slice_grid(bool f32, bool trans, int variant, int tiles, int kind = 0) {
  int grid = tiles;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
    const int cus = g_cus[dev].load(std::memory_order_relaxed);
    const int a = f32 ? 1 : 0, b = trans ? 1 : 0;
    const int occ = (kind == 1   ? g_occ_cx[a][b][variant]
                     : kind == 2 ? g_occ_emb[a][b][variant]
                                 : g_occ[a][b][variant])
                        .load(std::memory_order_relaxed);
    if (cus > 0 && occ > 0) grid = (int)std::min<int64_t>(tiles, (int64_t)cus * occ);
  }
  const int cap = g_slice_cap.load(std::memory_order_relaxed);
  if (cap > 0) grid = std::min(grid, cap);
  return grid;
}

template <typename T>
struct SliceLaunch {
  const T* src;
  int ld, rows, k, k_pad, gy, tiles;
  size_t slice;
  const void* aux;
  int8_t* out;
};

template <typename T, bool TR, int MODE, int PATH>
void launch_one(hipStream_t s, const SliceLaunch<T>& L, const CrtConsts& cc) {
  const int variant = MODE != 1 ? 0 : 1 + PATH;   // mode 2 has mode 0's resources
  const dim3 grid((unsigned)slice_grid(std::is_same<T, float>::value, TR, variant, L.tiles));
  hipLaunchKernelGGL((k_slices<T, TR, MODE, PATH>), grid, dim3(256), 0, s, L.src, L.ld, L.rows,
                     L.k, L.k_pad, L.gy, L.tiles, L.slice, L.aux, cc, L.out);
}

template <typename T, bool TR>
void launch_side(hipStream_t s, int mode, const SliceLaunch<T>& L, const CrtConsts& cc) {
  if (mode == 0) {
    launch_one<T, TR, 0, kAnyPath>(s, L, cc);
    return;
  }
  if (mode == 2) {
    launch_one<T, TR, 2, kAnyPath>(s, L, cc);
    return;
  }
  switch (residue_path(cc)) {
    case kLimbs2: launch_one<T, TR, 1, kLimbs2>(s, L, cc); break;
    case kLimbs3: launch_one<T, TR, 1, kLimbs3>(s, L, cc); break;
    case kSteps1: launch_one<T, TR, 1, kSteps1>(s, L, cc); break;
    case kSteps3: launch_one<T, TR, 1, kSteps3>(s, L, cc); break;
    default: launch_one<T, TR, 1, kSteps4>(s, L, cc); break;
  }
}

template <typename T, bool TR, int MODE, int PATH>
void launch_one_cx(hipStream_t s, const SliceLaunch<T>& L, const CrtConsts& cc) {
  const int variant = MODE != 1 ? 0 : 1 + PATH;
  const dim3 grid((unsigned)slice_grid(std::is_same<T, float>::value, TR, variant, L.tiles, 1));
  hipLaunchKernelGGL((k_slices_cx<T, TR, MODE, PATH>), grid, dim3(256), 0, s, L.src, L.ld, L.rows,
                     L.k, L.k_pad, L.gy, L.tiles, L.slice, L.aux, cc, L.out);
}

template <typename T, bool TR>
void launch_side_cx(hipStream_t s, int mode, const SliceLaunch<T>& L, const CrtConsts& cc) {
  if (mode == 2) {
    launch_one_cx<T, TR, 2, kAnyPath>(s, L, cc);
    return;
  }
  switch (residue_path(cc)) {
    case kLimbs2: launch_one_cx<T, TR, 1, kLimbs2>(s, L, cc); break;
    case kLimbs3: launch_one_cx<T, TR, 1, kLimbs3>(s, L, cc); break;
    case kSteps1: launch_one_cx<T, TR, 1, kSteps1>(s, L, cc); break;
    case kSteps3: launch_one_cx<T, TR, 1, kSteps3>(s, L, cc); break;
    default: launch_one_cx<T, TR, 1, kSteps4>(s, L, cc); break;
  }
}

template <typename T>
void launch_t(hipStream_t s, int mode, bool trans, const T* src, int ld, int rows, int k,
              int rows_pad, int k_pad, const uint64_t* bits, const int* shift, const CrtConsts& cc,
              int8_t* out, bool cx = false) {
  SliceLaunch<T> L;
  L.src = src;
  L.ld = ld;
  L.rows = rows;
  L.k = k;
  L.k_pad = k_pad;
  L.gy = mode != 1 ? rows_pad / kTR : cdiv_i(rows, kTR);
  L.tiles = (k_pad / kTK) * L.gy;
  L.slice = (size_t)rows_pad * k_pad;
  L.aux = mode != 1 ? (const void*)bits : (const void*)shift;
  L.out = out;
  if (L.tiles <= 0) return;
  if (cx) {
    if (trans)
      launch_side_cx<T, true>(s, mode, L, cc);
    else
      launch_side_cx<T, false>(s, mode, L, cc);
  } else if (trans) {
    launch_side<T, true>(s, mode, L, cc);
  } else {
    launch_side<T, false>(s, mode, L, cc);
  }
}

template <typename T, bool TR, int MODE, int PATH>
void launch_group_one(hipStream_t s, const ProbDesc* P, const BlockRef* map, int blocks,
                      const CrtConsts* ctab) {
  const int variant = kGrouped + (MODE == 0 ? 0 : 1 + PATH);
  const dim3 g((unsigned)slice_grid(std::is_same<T, float>::value, TR, variant, blocks)), b(256);
  hipLaunchKernelGGL((kg_slices<T, TR, MODE, PATH>), g, b, 0, s, P, map, blocks, ctab);
}

template <typename T, bool TR>
void group_slices_t(hipStream_t s, int mode, int path, const ProbDesc* P, const BlockRef* map,
                    int blocks, const CrtConsts* ctab) {
  if (mode == 0) {
    launch_group_one<T, TR, 0, kAnyPath>(s, P, map, blocks, ctab);
    return;
  }
  switch (path) {
    case kLimbs2: launch_group_one<T, TR, 1, kLimbs2>(s, P, map, blocks, ctab); break;
    case kLimbs3: launch_group_one<T, TR, 1, kLimbs3>(s, P, map, blocks, ctab); break;
    case kSteps1: launch_group_one<T, TR, 1, kSteps1>(s, P, map, blocks, ctab); break;
    case kSteps3: launch_group_one<T, TR, 1, kSteps3>(s, P, map, blocks, ctab); break;
    case kSteps4: launch_group_one<T, TR, 1, kSteps4>(s, P, map, blocks, ctab); break;
    default: launch_group_one<T, TR, 1, kAnyPath>(s, P, map, blocks, ctab); break;
  }
}

}  // namespace

std::atomic<int> g_slice_cap{0};

void init_slice_launch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  fill_occ<double, true>();
  fill_occ<double, false>();
  fill_occ<float, true>();
  fill_occ<float, false>();
  g_cus[dev].store(cus, std::memory_order_relaxed);
}

int group_residue_path(const CrtConsts* const* cc, int count) {
  int path = -1;
  for (int q = 0; q < count; ++q) {
    const int r = residue_path(*cc[q]);
    if (path >= 0 && r != path) return kAnyPath;
    path = r;
  }
  return path < 0 ? kAnyPath : path;
}

void launch_group_slices(hipStream_t s, Prec pr, int mode, bool aside, int path,
                         const ProbDesc* P, const BlockRef* map, int blocks,
                         const CrtConsts* ctab) {
  if (blocks <= 0) return;
  if (path < 0 || path > kAnyPath) path = kAnyPath;
  if (pr == Prec::F64) {
    if (aside)
      group_slices_t<double, true>(s, mode, path, P, map, blocks, ctab);
    else
      group_slices_t<double, false>(s, mode, path, P, map, blocks, ctab);
  } else {
    if (aside)
      group_slices_t<float, true>(s, mode, path, P, map, blocks, ctab);
    else
      group_slices_t<float, false>(s, mode, path, P, map, blocks, ctab);
  }
}

void launch_plan_slices(hipStream_t s, Prec pr, bool trans, const void* src, int ld, int rows,
                        int k, int rows_pad, int k_pad, const uint64_t* bits, uint16_t* out,
                        double* partial) {
  // Four workgroups per CU (33 KB of LDS each) walk the tiles.
  const int64_t tiles = (int64_t)(k_pad / kPlanTile) * (rows_pad / kPlanTile);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices)
    cus = g_cus[dev].load(std::memory_order_relaxed);
  if (tiles <= 0) return;
  const int64_t cap = 4 * (int64_t)(cus > 0 ? cus : 256);
  const dim3 grid((unsigned)(tiles < cap ? tiles : cap));
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

namespace {

template <typename T, bool TR, int MODE, int PATH>
void emb_one(hipStream_t s, const T* src, int ld, int rows, int k, int kh, int gy, int tiles,
             int half, size_t slice, const void* aux, const CrtConsts& cc, int8_t* out) {
  const int variant = MODE == 0 ? 0 : 1 + PATH;
  const dim3 grid((unsigned)slice_grid(std::is_same<T, float>::value, TR, variant, tiles, 2));
  hipLaunchKernelGGL((k_slices_emb<T, TR, MODE, PATH>), grid, dim3(256), 0, s, src, ld, rows, k,
                     kh, gy, tiles, half, slice, aux, cc, out);
}

template <typename T, bool TR>
void emb_side(hipStream_t s, int mode, const T* src, int ld, int rows, int k, int kh, int rows_pad,
              int half, const uint64_t* bits, const int* shift, const CrtConsts& cc, int8_t* out) {
  // mode 0 covers the padding rows (their bars must be zero); mode 1 only
  // the tiles of real rows.  On the A side the tiles cover the first half.
  const int span = TR ? half : rows_pad;
  const int gy = mode == 0 ? span / kTR : cdiv_i(rows, kTR);
  const int tiles = (kh / kTK) * gy;
  const size_t slice = (size_t)rows_pad * 2 * kh;
  if (tiles <= 0) return;
  if (mode == 0) {
    emb_one<T, TR, 0, kAnyPath>(s, src, ld, rows, k, kh, gy, tiles, half, slice, bits, cc, out);
    return;
  }
  switch (residue_path(cc)) {
    case kLimbs2: emb_one<T, TR, 1, kLimbs2>(s, src, ld, rows, k, kh, gy, tiles, half, slice, shift, cc, out); break;
    case kLimbs3: emb_one<T, TR, 1, kLimbs3>(s, src, ld, rows, k, kh, gy, tiles, half, slice, shift, cc, out); break;
    case kSteps1: emb_one<T, TR, 1, kSteps1>(s, src, ld, rows, k, kh, gy, tiles, half, slice, shift, cc, out); break;
    case kSteps3: emb_one<T, TR, 1, kSteps3>(s, src, ld, rows, k, kh, gy, tiles, half, slice, shift, cc, out); break;
    default: emb_one<T, TR, 1, kSteps4>(s, src, ld, rows, k, kh, gy, tiles, half, slice, shift, cc, out); break;
  }
}

}  // namespace

void launch_slices_embed(hipStream_t s, Prec pr, int mode, bool aside, const void* src, int ld,
                         int rows, int k, int kh, int rows_pad, int half, const uint64_t* bits,
                         const int* shift, const CrtConsts& cc, int8_t* out) {
  if (mode != 0 && mode != 1) return;
  if (pr == Prec::F64) {
    if (aside)
      emb_side<double, true>(s, mode, (const double*)src, ld, rows, k, kh, rows_pad, half, bits,
                             shift, cc, out);
    else
      emb_side<double, false>(s, mode, (const double*)src, ld, rows, k, kh, rows_pad, 0, bits,
                              shift, cc, out);
  } else {
    if (aside)
      emb_side<float, true>(s, mode, (const float*)src, ld, rows, k, kh, rows_pad, half, bits,
                            shift, cc, out);
    else
      emb_side<float, false>(s, mode, (const float*)src, ld, rows, k, kh, rows_pad, 0, bits, shift,
                             cc, out);
  }
}

void launch_slices_complex(hipStream_t s, Prec pr, int mode, bool trans, const void* src, int ld,
                           int rows, int k, int rows_pad, int k_pad, const uint64_t* bits,
                           const int* shift, const CrtConsts& cc, int8_t* out) {
  if (mode != 1 && mode != 2) return;
  if (pr == Prec::F64)
    launch_t<double>(s, mode, trans, (const double*)src, ld, rows, k, rows_pad, k_pad, bits, shift,
                     cc, out, true);
  else
    launch_t<float>(s, mode, trans, (const float*)src, ld, rows, k, rows_pad, k_pad, bits, shift,
                    cc, out, true);
}

}  // namespace oz2
