// INT8 x INT8 -> INT32 matrix-core products (CDNA4 v_mfma_i32_32x32x32_i8):
//   epi 0: the N residue products C'_l = A'_l B'_l of Algorithm 3 with the
//          reduction W_l = mod(C'_l, p_l) fused into the epilogue;
//   epi 1: the scaling product Cbar = Abar Bbar of Algorithm 2, of which only
//          the row and column maxima are kept (atomicMax, order-free).
//
// Operands are K-major INT8 slices (k contiguous), zero padded, so the kernel
// needs no bounds checks:  D[x][y] = sum_h X[x][h] Y[y][h].  The library
// passes X = B-side slice (x = output column j) and Y = A-side slice
// (y = output row i), so that in the MFMA accumulator layout consecutive
// lanes hold consecutive i and W_l[j][i] stores are contiguous.
//
// Tiling: a 256-thread workgroup (4 waves as 2 x 2) computes a BX x BY tile;
// each wave owns (BX/2) x (BY/2) as (BX/64) x (BY/64) blocks of 32 x 32.
// K advances BK bytes per stage through a double-buffered LDS tile with rows
// padded by 16 bytes (conflict-free 16-byte fragment reads); global loads of
// the next stage are issued before the MFMAs of the current one.
//
// Accumulator layout of the 32x32x32 MFMA (lane l, register r):
//   row (X side) = 8*(r/4) + 4*(l/32) + r%4,   column (Y side) = l%32.
#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// mod(x, p) of an INT32 product as an INT8 value (Section 1.2).  For odd p
// the FP64 quotient x * (1/p) is within 2^-25 of x/p, which is never within
// 1/(2p) of a half-integer, so rint gives round(x/p) exactly.  For p = 256
// the low byte is the two's-complement wrap of Section 3.1.
__device__ inline int mod_i32(int x, int p, double pinv) {
  if (p == 256) return (int)(int8_t)(x & 0xFF);
  const double q = rint((double)x * pinv);
  return x - (int)q * p;
}

template <int BX, int BY, int BK, int EPI>
__global__ __launch_bounds__(256, 1) void k_gemm_i8(const int8_t* __restrict__ X, size_t sx,
                                                    const int8_t* __restrict__ Y, size_t sy,
                                                    int tiles_x, int k_pad, CrtConsts cc,
                                                    int8_t* __restrict__ W, size_t sw, int ldw,
                                                    int* __restrict__ xmax, int* __restrict__ ymax) {
  constexpr int WX = BX / 2, WY = BY / 2;
  constexpr int TX = WX / 32, TY = WY / 32;
  constexpr int LDK = BK + 16;
  constexpr int CPR = BK / 16;                    // 16-byte chunks per row
  constexpr int CHX = BX * CPR / 256, CHY = BY * CPR / 256;
  static_assert(CHX * 256 == BX * CPR && CHY * 256 == BY * CPR, "tile / thread mismatch");
  __shared__ __attribute__((aligned(16))) int8_t lds[2][(BX + BY) * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wx = wave >> 1, wy = wave & 1;
  const int z = blockIdx.y;
  const int tile = blockIdx.x;
  const int x0 = (tile % tiles_x) * BX, y0 = (tile / tiles_x) * BY;
  const int8_t* Xz = X + (size_t)z * sx + (size_t)x0 * k_pad;
  const int8_t* Yz = Y + (size_t)z * sy + (size_t)y0 * k_pad;

  v4i rx[CHX], ry[CHY];
  auto gload = [&](int k0) {
#pragma unroll
    for (int c = 0; c < CHX; ++c) {
      const int idx = tid + 256 * c, row = idx / CPR, col = idx % CPR;
      rx[c] = *reinterpret_cast<const v4i*>(Xz + (size_t)row * k_pad + k0 + col * 16);
    }
#pragma unroll
    for (int c = 0; c < CHY; ++c) {
      const int idx = tid + 256 * c, row = idx / CPR, col = idx % CPR;
      ry[c] = *reinterpret_cast<const v4i*>(Yz + (size_t)row * k_pad + k0 + col * 16);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CHX; ++c) {
      const int idx = tid + 256 * c, row = idx / CPR, col = idx % CPR;
      *reinterpret_cast<v4i*>(&lds[buf][row * LDK + col * 16]) = rx[c];
    }
#pragma unroll
    for (int c = 0; c < CHY; ++c) {
      const int idx = tid + 256 * c, row = idx / CPR, col = idx % CPR;
      *reinterpret_cast<v4i*>(&lds[buf][(BX + row) * LDK + col * 16]) = ry[c];
    }
  };

  v16i acc[TX][TY];
#pragma unroll
  for (int a = 0; a < TX; ++a)
#pragma unroll
    for (int b = 0; b < TY; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  const int KT = k_pad / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int frow = lane & 31, fk = (lane >> 5) * 16;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * BK);
    const int8_t* Ls = lds[cur];
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      v4i a[TX], b[TY];
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
        a[tx] = *reinterpret_cast<const v4i*>(Ls + (wx * WX + tx * 32 + frow) * LDK + kk * 32 + fk);
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
        b[ty] = *reinterpret_cast<const v4i*>(Ls + (BX + wy * WY + ty * 32 + frow) * LDK + kk * 32 + fk);
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty)
          acc[tx][ty] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tx], b[ty], acc[tx][ty], 0, 0, 0);
    }
    if (kt + 1 < KT) lstore(cur ^ 1);
    __syncthreads();
  }

  const int xb = x0 + wx * WX, yb = y0 + wy * WY;
  if (EPI == 0) {
    const int p = cc.p[z];
    const double pinv = cc.pinv[z];
    int8_t* Wz = W + (size_t)z * sw;
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int x = xb + tx * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int y = yb + ty * 32 + (lane & 31);
          Wz[(size_t)x * ldw + y] = (int8_t)mod_i32(acc[tx][ty][r], p, pinv);
        }
  } else {
    // max over x for each y (row maxima of Cbar when y = i)
#pragma unroll
    for (int ty = 0; ty < TY; ++ty) {
      int mv = 0;
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int r = 0; r < 16; ++r) mv = max(mv, acc[tx][ty][r]);
      mv = max(mv, __shfl_xor(mv, 32));
      if (lane < 32) atomicMax(&ymax[yb + ty * 32 + lane], mv);
    }
    // max over y for each x
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int mv = 0;
#pragma unroll
        for (int ty = 0; ty < TY; ++ty) mv = max(mv, acc[tx][ty][r]);
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) mv = max(mv, __shfl_xor(mv, off));
        if ((lane & 31) == 0)
          atomicMax(&xmax[xb + tx * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)], mv);
      }
  }
}

}  // namespace

void launch_gemm_i8(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                    int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                    size_t sw, int ldw, int* xmax, int* ymax) {
  constexpr int BX = 128, BY = 128, BK = 128;
  const int tiles_x = nx_pad / BX, tiles_y = ny_pad / BY;
  dim3 grid((unsigned)(tiles_x * tiles_y), (unsigned)nz);
  if (epi == 0)
    hipLaunchKernelGGL((k_gemm_i8<BX, BY, BK, 0>), grid, dim3(256), 0, s, X, sx, Y, sy, tiles_x,
                       k_pad, cc, W, sw, ldw, xmax, ymax);
  else
    hipLaunchKernelGGL((k_gemm_i8<BX, BY, BK, 1>), grid, dim3(256), 0, s, X, sx, Y, sy, tiles_x,
                       k_pad, cc, W, sw, ldw, xmax, ymax);
}

}  // namespace oz2
