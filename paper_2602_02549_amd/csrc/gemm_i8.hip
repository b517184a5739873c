// INT8 x INT8 -> INT32 matrix-core products (CDNA4 v_mfma_i32_32x32x32_i8):
//   epi 0: the N residue products C'_l = A'_l B'_l of Algorithm 3 with the
//          reduction W_l = mod(C'_l, p_l) fused into the epilogue;
//   epi 1: the scaling product Cbar = Abar Bbar of Algorithm 2, of which only
//          the row and column maxima are kept (atomicMax, order-free).
//
// Operands are K-major INT8 slices (k contiguous), zero padded, so the kernel
// needs no bounds checks:  D[x][y] = sum_h X[x][h] Y[y][h], with X the A side
// (x = output row i) and Y the B side (y = output column j).  In the MFMA
// accumulator layout a lane holds 4 consecutive x for one y, so the W_l bytes
// of 4 consecutive rows i are packed into one 32-bit store of the
// column-major W_l[j][i].
//
// Tiling: a 256-thread workgroup (4 waves as 2 x 2) computes a BX x BY tile;
// each wave owns (BX/2) x (BY/2) as (BX/64) x (BY/64) blocks of 32 x 32
// (accumulators live in AGPRs).  K advances 64 bytes per stage through a ring
// of S LDS stage buffers filled by direct global->LDS copies issued S-1
// stages ahead, so HBM/L2 latency is covered by the MFMAs of S-1 stages.
//
// Workgroup order: the hardware deals workgroups round-robin to the 8 XCDs;
// the linear id is remapped so each XCD works on a contiguous range of
// tiles, and tiles are walked in groups of GROUP rows of tiles so that the
// workgroups resident on one XCD share A- and B-panels in its L2.
//
// Accumulator layout of the 32x32x32 MFMA (lane l, register r):
//   row (X side) = 8*(r/4) + 4*(l/32) + r%4,   column (Y side) = l%32.
#include <cstdint>
#include <type_traits>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kXcds = 8;

// mod(x, p) of an INT32 product as an INT8 value (Section 1.2).  For odd p
// the FP64 quotient x * (1/p) is within 2^-25 of x/p, which is never within
// 1/(2p) of a half-integer, so rint gives round(x/p) exactly.  For p = 256
// the low byte is the two's-complement wrap of Section 3.1.
__device__ inline int mod_i32(int x, int p, double pinv) {
  if (p == 256) return (int)(int8_t)(x & 0xFF);
  const double q = rint((double)x * pinv);
  return x - (int)q * p;
}

typedef __attribute__((address_space(3))) int8_t lds_i8_t;

// One wave-wide direct global->LDS copy (CDNA4 global_load_lds_dwordx4):
// lane l copies 16 bytes from its address g to LDS byte M0 + 16 l.  Issued as
// inline asm so the compiler's wait-count insertion does not treat every LDS
// read as depending on every copy in flight; the kernel waits explicitly.
__device__ inline void dma16(const void* g, uint32_t lds_addr) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(g), "s"(lds_addr)
               : "memory", "m0");
}

__device__ inline uint32_t lds_addr(const int8_t* p) {
  return (uint32_t)(uintptr_t)(lds_i8_t*)p;
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding).
template <int V>
__device__ inline void wait_vmcnt() {
  static_assert(V >= 0 && V < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((V & 0xF) | (((V >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8));
}

// Main loop structure (BK = 64, S LDS stages filled by global_load_lds):
// each stage buffer holds the X tile then the Y tile as rows of 64 bytes;
// the four 16-byte chunks of row r sit at chunk positions c ^ swz(r),
// swz(r) = (r >> 1) & 3, so the 16-byte fragment reads of 8 consecutive rows
// hit distinct bank groups.  One wave instruction moves 16 rows (1 KB).
template <int BX, int BY, int S, int EPI>
__global__ __launch_bounds__(256, 1) void k_gemm_i8(const int8_t* __restrict__ X, size_t sx,
                                                    const int8_t* __restrict__ Y, size_t sy,
                                                    int tiles_x, int tiles_y, int nz, int k_pad,
                                                    CrtConsts cc, int8_t* __restrict__ W, size_t sw,
                                                    int ldw, int* __restrict__ xmax,
                                                    int* __restrict__ ymax) {
  constexpr int BK = 64;
  constexpr int WX = BX / 2, WY = BY / 2;
  constexpr int TX = WX / 32, TY = WY / 32;
  constexpr int IX = BX / 16 / 4, IY = BY / 16 / 4;   // DMA instructions per wave per stage
  constexpr int LPS = IX + IY;
  constexpr int STAGE = (BX + BY) * BK;
  constexpr int GROUP = 8;
  static_assert(S >= 3 && S <= 4, "stages");
  __shared__ __attribute__((aligned(1024))) int8_t lds0[STAGE];
  __shared__ __attribute__((aligned(1024))) int8_t lds1[STAGE];
  __shared__ __attribute__((aligned(1024))) int8_t lds2[STAGE];
  __shared__ __attribute__((aligned(1024))) int8_t lds3[S == 4 ? STAGE : 16];

  // ---- workgroup -> (slice z, tile) ------------------------------------
  const int total = tiles_x * tiles_y * nz;
  int bid = blockIdx.x;
  {
    const int xcd = bid % kXcds, loc = bid / kXcds;
    const int per = total / kXcds, extra = total % kXcds;
    bid = xcd * per + min(xcd, extra) + loc;
  }
  const int per_slice = tiles_x * tiles_y;
  const int z = bid / per_slice;
  int t = bid % per_slice;
  const int group_span = GROUP * tiles_y;
  const int g = t / group_span;
  const int gx0 = g * GROUP;
  const int gsz = min(GROUP, tiles_x - gx0);
  t -= g * group_span;
  const int tx_ = gx0 + t % gsz, ty_ = t / gsz;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wx = wave >> 1, wy = wave & 1;
  const int x0 = tx_ * BX, y0 = ty_ * BY;

  // DMA source pointers: instruction q of this wave covers rows 16q..16q+15.
  const int drow = lane >> 2;
  const int dchunk = (lane & 3) ^ ((lane >> 3) & 3);
  const int8_t* xsrc = X + (size_t)z * sx + (size_t)(x0 + wave * IX * 16 + drow) * k_pad + dchunk * 16;
  const int8_t* ysrc = Y + (size_t)z * sy + (size_t)(y0 + wave * IY * 16 + drow) * k_pad + dchunk * 16;
  const size_t rowstep = (size_t)16 * k_pad;

  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto issue = [&](int8_t* buf, int k0) {
    const uint32_t base = lds_addr(buf);
#pragma unroll
    for (int q = 0; q < IX; ++q)
      dma16(xsrc + q * rowstep + k0, base + (uint32_t)((wave_u * IX + q) * 1024));
#pragma unroll
    for (int q = 0; q < IY; ++q)
      dma16(ysrc + q * rowstep + k0, base + (uint32_t)(BX * BK + (wave_u * IY + q) * 1024));
  };

  v16i acc[TX][TY];
#pragma unroll
  for (int a = 0; a < TX; ++a)
#pragma unroll
    for (int b = 0; b < TY; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  // fragment addressing: lane reads row frow of a 32-row block, k chunk 2kk + lane/32
  const int frow = lane & 31;
  const int swz = (frow >> 1) & 3;
  const int fo0 = frow * BK + ((0 + (lane >> 5)) ^ swz) * 16;
  const int fo1 = frow * BK + ((2 + (lane >> 5)) ^ swz) * 16;
  auto compute = [&](const int8_t* buf) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int fo = kk ? fo1 : fo0;
      v4i a[TX], b[TY];
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
        a[tx] = *reinterpret_cast<const v4i*>(buf + (wx * WX + tx * 32) * BK + fo);
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
        b[ty] = *reinterpret_cast<const v4i*>(buf + (BX + wy * WY + ty * 32) * BK + fo);
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty)
          acc[tx][ty] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tx], b[ty], acc[tx][ty], 0, 0, 0);
    }
  };
  int8_t* bufs[4] = {lds0, lds1, lds2, lds3};

  const int KT = k_pad / BK;
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < KT) issue(bufs[s], s * BK);

  // One step per k stage; the loop is unrolled S times so every buffer is a
  // static object (the compiler then waits only for the DMA it reads).
  auto step = [&](auto sc, int kt) {
    constexpr int s = decltype(sc)::value;
    if (kt + S - 2 < KT)
      wait_vmcnt<(S - 2) * LPS>();
    else
      wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (kt + S - 1 < KT) issue(bufs[(s + S - 1) % S], (kt + S - 1) * BK);
    compute(bufs[s]);
  };
  for (int kt = 0; kt < KT; kt += S) {
    step(std::integral_constant<int, 0>{}, kt);
    if (kt + 1 < KT) step(std::integral_constant<int, 1>{}, kt + 1);
    if (kt + 2 < KT) step(std::integral_constant<int, 2>{}, kt + 2);
    if (S == 4 && kt + 3 < KT) step(std::integral_constant<int, (S == 4 ? 3 : 0)>{}, kt + 3);
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
        for (int r4 = 0; r4 < 4; ++r4) {
          const int x = xb + tx * 32 + 8 * r4 + 4 * (lane >> 5);
          const int y = yb + ty * 32 + (lane & 31);
          const uint32_t w = (uint32_t)(mod_i32(acc[tx][ty][4 * r4 + 0], p, pinv) & 0xFF) |
                             ((uint32_t)(mod_i32(acc[tx][ty][4 * r4 + 1], p, pinv) & 0xFF) << 8) |
                             ((uint32_t)(mod_i32(acc[tx][ty][4 * r4 + 2], p, pinv) & 0xFF) << 16) |
                             ((uint32_t)(mod_i32(acc[tx][ty][4 * r4 + 3], p, pinv) & 0xFF) << 24);
          *reinterpret_cast<uint32_t*>(Wz + (size_t)y * ldw + x) = w;
        }
  } else {
    // max over x for each y
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

template <int BX, int BY, int S>
void launch_cfg(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                size_t sw, int ldw, int* xmax, int* ymax) {
  const int tiles_x = nx_pad / BX, tiles_y = ny_pad / BY;
  dim3 grid((unsigned)(tiles_x * tiles_y * nz));
  if (epi == 0)
    hipLaunchKernelGGL((k_gemm_i8<BX, BY, S, 0>), grid, dim3(256), 0, s, X, sx, Y, sy, tiles_x,
                       tiles_y, nz, k_pad, cc, W, sw, ldw, xmax, ymax);
  else
    hipLaunchKernelGGL((k_gemm_i8<BX, BY, S, 1>), grid, dim3(256), 0, s, X, sx, Y, sy, tiles_x,
                       tiles_y, nz, k_pad, cc, W, sw, ldw, xmax, ymax);
}

}  // namespace

void launch_gemm_i8(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                    int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                    size_t sw, int ldw, int* xmax, int* ymax) {
  // 256 x 256 tiles when they give at least ~2 workgroups per CU, else 128 x 128.
  const long big_tiles = (long)(nx_pad / 256) * (ny_pad / 256) * nz;
  if (nx_pad % 256 == 0 && ny_pad % 256 == 0 && big_tiles >= 512)
    launch_cfg<256, 256, 4>(s, epi, X, sx, Y, sy, nx_pad, ny_pad, k_pad, nz, cc, W, sw, ldw, xmax,
                             ymax);
  else
    launch_cfg<128, 128, 4>(s, epi, X, sx, Y, sy, nx_pad, ny_pad, k_pad, nz, cc, W, sw, ldw,
                              xmax, ymax);
}

}  // namespace oz2
