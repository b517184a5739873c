// INT8 x INT8 -> INT32 matrix-core products (CDNA4 v_mfma_i32_32x32x32_i8):
//   epi 0: the N residue products C'_l = A'_l B'_l of Algorithm 3 with the
//          reduction W_l = mod(C'_l, p_l) fused into the epilogue;
//   epi 1: the scaling product Cbar = Abar Bbar of Algorithm 2, of which only
//          the row and column maxima are kept (atomicMax, order-free);
//   epi 3: epi 1 plus one byte per entry, Cbar_ij != 0 (the planner's
//          indicator of (|A||B|)_ij > 0);
//   epi 4: the raw INT32 accumulators C'_l (stage dumps only).
//
// Operands are K-major INT8 slices (k contiguous), zero padded, so the kernel
// needs no bounds checks:  D[x][y] = sum_h X[x][h] Y[y][h], with X the A side
// (x = output row i) and Y the B side (y = output column j).  In the MFMA
// accumulator layout a lane holds 4 consecutive x for one y, so the W_l bytes
// of 4 consecutive rows i are packed into one 32-bit store of the
// column-major W_l[j][i].
//
// Tiling: a workgroup of NWX x NWY waves computes a BX x BY tile; each wave
// owns (BX/NWX) x (BY/NWY) as blocks of 32 x 32.  A 256 x 256 tile runs 8
// waves (4 x 2, each 64 x 128: two waves per SIMD, so one wave's MFMAs
// overlap the other's LDS reads and barrier waits), a 128 x 128 tile 4 waves
// (2 x 2) with two workgroups per CU.  K advances in groups of 128
// bytes through two LDS group buffers: direct global->LDS copies fill one
// (every 128-byte line of an operand row requested as one unit) while the
// MFMAs consume the other.  BF16 operands (the planner's lower bound of
// |A||B|) run through the same loop, counting k in bytes.
//
// Workgroup order: the hardware deals workgroups round-robin to the 8 XCDs;
// the linear id is remapped so each XCD works on a contiguous range of
// tiles, and tiles are walked in groups of GROUP rows of tiles so that the
// workgroups resident on one XCD share A- and B-panels in its L2.
//
// Accumulator layout of the 32x32x32 MFMA (lane l, register r):
//   row (X side) = 8*(r/4) + 4*(l/32) + r%4,   column (Y side) = l%32.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <type_traits>

#include "ozaki2_internal.h"
#include "small_mod.h"

namespace oz2 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));

constexpr int kXcds = 8;
constexpr int kFoldGroups = (1 << 17) / 128;   // 128-k groups per 2^17 of k

// mod(x, p) of an INT32 product as an INT8 value (Section 1.2), odd p: the
// FP64 quotient x * (1/p) is within 2^-25 of x/p, which is never within
// 1/(2p) of a half-integer, so rint gives round(x/p) exactly and one fma
// gives x - round(x/p) p exactly.  (p = 256 takes the low byte, the
// two's-complement wrap of Section 3.1, in the caller.)
__device__ inline int mod_odd(int x, double p, double pinv) {
  const double xd = (double)x;
  return (int)fma(-rint(xd * pinv), p, xd);
}

__device__ inline uint32_t pack_bytes(int a, int b, int c, int d) {
  return (uint32_t)(a & 0xFF) | ((uint32_t)(b & 0xFF) << 8) | ((uint32_t)(c & 0xFF) << 16) |
         ((uint32_t)(d & 0xFF) << 24);
}

typedef __attribute__((address_space(3))) int8_t lds_i8_t;

// One wave-wide direct global->LDS copy (CDNA4 global_load_lds_dwordx4):
// lane l copies 16 bytes from its address g to LDS byte M0 + 16 l.  Issued as
// inline asm so the compiler's wait-count insertion does not treat every LDS
// read as depending on every copy in flight; the kernel waits explicitly.
// M0 is saved in a scratch SGPR and restored, so no value the compiler keeps
// in M0 is disturbed.
__device__ inline void dma16(const void* g, uint32_t lds_addr) {
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\t"
      "global_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(g), "s"(lds_addr)
      : "memory");
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

// Chunk swizzle of an LDS row (128 bytes of k, 32 banks apart): chunk c of
// row r is stored at position c ^ swz(r), so that the 16-byte fragment reads
// of rows r..r+15 land in distinct bank groups (64 banks).
__device__ inline int swz(int r) { return (r >> 1) & 7; }

// Main loop structure: k advances in groups of 128 bytes; two groups (128 KB
// for a 256x256 tile) are resident in LDS.  The copies of group g+1 (direct
// global->LDS, every 128-byte line requested as one unit) run while the
// MFMAs consume group g.  A group buffer holds the X tile then the Y tile as
// rows of 128 bytes.  `bid` is the workgroup's index among the `launched`
// workgroups of this product (launched >= tiles_x * tiles_y * nz * nsplit;
// the surplus exits at once).  Split-k: with nsplit > 1, workgroup index
// sidx = bid / (tiles * nz) takes the k-groups [sidx G / nsplit,
// (sidx + 1) G / nsplit) of the G = k_pad / 128 (nsplit <= G), and its
// epilogue writes slice sidx * nz + z of W (EPI 0: mod p_z of its partial
// sum; EPI 4: the INT32 partial sum); the caller reduces the partials.
// SPLIT selects that build; without it nsplit is 1 and the k loop is the
// plain one from group 0 (a dynamic start cost 2% at 8192^3).
template <int BX, int BY, int NWX, int NWY, int EPI, bool BF16, bool FOLD, bool SPLIT = false>
__device__ __forceinline__ void gemm_body(const int8_t* __restrict__ X, size_t sx,
                                          const int8_t* __restrict__ Y, size_t sy, int tiles_x,
                                          int tiles_y, int nz, int k_pad, const CrtConsts& cc,
                                          int8_t* __restrict__ W, size_t sw, int ldw,
                                          int* __restrict__ xmax, int* __restrict__ ymax, int bid,
                                          int launched, int nsplit = 1) {
  constexpr int BK = 128;                        // bytes of k per LDS row (one group)
  constexpr int NW = NWX * NWY;                  // waves
  constexpr int WX = BX / NWX, WY = BY / NWY;
  constexpr int TX = WX / 32, TY = WY / 32;
  constexpr int CPR = BK / 16;                   // 16-byte chunks per LDS row
  constexpr int RPI = 1024 / BK;                 // rows per copy instruction
  constexpr int IX = BX / RPI / NW, IY = BY / RPI / NW;
  // Each wave copies IX (IY) instructions of RPI rows; the chunk swizzle
  // repeats every 16 rows and the even/odd instruction offsets below assume
  // that every wave's share starts at a multiple of 16 rows.
  static_assert(IX % 2 == 0 && IY % 2 == 0 && WX % 32 == 0 && WY % 32 == 0, "tile / wave shape");
  constexpr int GROUP_BYTES = (BX + BY) * BK;    // one 128-k group
  constexpr int GROUP = 8;
  __shared__ __attribute__((aligned(1024))) int8_t lds[2 * GROUP_BYTES];

  // ---- workgroup -> (slice z, tile) ------------------------------------
  if constexpr (!SPLIT) nsplit = 1;
  const int total = tiles_x * tiles_y * nz * nsplit;
  {
    const int xcd = bid % kXcds, loc = bid / kXcds;
    const int per = launched / kXcds, extra = launched % kXcds;
    bid = xcd * per + min(xcd, extra) + loc;
  }
  if (bid >= total) return;   // whole workgroup, before any barrier
  const int per_slice = tiles_x * tiles_y;
  const int sidx = SPLIT ? bid / (per_slice * nz) : 0;
  bid -= sidx * per_slice * nz;
  const int z = bid / per_slice;
  int t = bid % per_slice;
  const int group_span = GROUP * tiles_y;
  const int g = t / group_span;
  const int gx0 = g * GROUP;
  const int gsz = min(GROUP, tiles_x - gx0);
  t -= g * group_span;
  const int tx_ = gx0 + t % gsz, ty_ = t / gsz;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wx = wave / NWY, wy = wave % NWY;
  const int x0 = tx_ * BX, y0 = ty_ * BY;

  // Copy instruction q of this wave covers rows RPI*q .. RPI*q + RPI - 1 of
  // its share; lane l takes row RPI*q + l/CPR and stores LDS chunk l%CPR,
  // which holds k-chunk (l%CPR) ^ swz(row).
  const int lr = lane / CPR, slot = lane % CPR;
  const int ch_e = (slot ^ swz(lr)) * 16, ch_o = (slot ^ swz(RPI + lr)) * 16;
  const int8_t* xsrc = X + (size_t)(x0 + wave * IX * RPI + lr) * k_pad;
  const int8_t* ysrc = Y + (size_t)(y0 + wave * IY * RPI + lr) * k_pad;
  const size_t rowstep = (size_t)RPI * k_pad;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);

  // The copies of one group: the X rows (issue_x) and the Y rows (issue_y).
  auto issue_x = [&](int8_t* buf, int z, int k0) {
    const uint32_t b = lds_addr(buf);
    const int8_t* xs = xsrc + (size_t)z * sx + k0;
#pragma unroll
    for (int q = 0; q < IX; ++q)
      dma16(xs + q * rowstep + ((q & 1) ? ch_o : ch_e), b + (uint32_t)((wave_u * IX + q) * 1024));
  };
  auto issue_y = [&](int8_t* buf, int z, int k0) {
    const uint32_t b = lds_addr(buf);
    const int8_t* ys = ysrc + (size_t)z * sy + k0;
#pragma unroll
    for (int q = 0; q < IY; ++q)
      dma16(ys + q * rowstep + ((q & 1) ? ch_o : ch_e),
            b + (uint32_t)(BX * BK + (wave_u * IY + q) * 1024));
  };

  using AccT = typename std::conditional<BF16, v16f, v16i>::type;
  AccT acc[TX][TY];
#pragma unroll
  for (int a = 0; a < TX; ++a)
#pragma unroll
    for (int b = 0; b < TY; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  // fragment offsets of the four 32-k sub-steps j of a group: lane reads row
  // frow of a 32-row block, k chunk 2j + lane/32 of the group
  const int frow = lane & 31;
  int fo[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) fo[j] = frow * BK + (((2 * j + (lane >> 5)) ^ swz(frow)) * 16);
  auto load_frags = [&](const int8_t* buf, int j, v4i (&a)[TX], v4i (&b)[TY]) {
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
      a[tx] = *reinterpret_cast<const v4i*>(buf + (wx * WX + tx * 32) * BK + fo[j]);
#pragma unroll
    for (int ty = 0; ty < TY; ++ty)
      b[ty] = *reinterpret_cast<const v4i*>(buf + (BX + wy * WY + ty * 32) * BK + fo[j]);
  };
  auto mfmas = [&](const v4i (&a)[TX], const v4i (&b)[TY]) {
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
        if constexpr (BF16)
          acc[tx][ty] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(v8bf16, a[tx]), __builtin_bit_cast(v8bf16, b[ty]), acc[tx][ty], 0,
              0, 0);
        else
          acc[tx][ty] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tx], b[ty], acc[tx][ty], 0, 0, 0);
  };

  const int xb = x0 + wx * WX, yb = y0 + wy * WY;
  // Per 32 x 32 block, lane l holds rows {0-3, 8-11, 16-19, 24-27} + 4 (l/32)
  // of column l%32, packed as 4 dwords R0..R3 (one byte per row).  Swapping
  // R0<->R2 and R1<->R3 between lanes l and l+32 (v_permlane32_swap) leaves
  // rows 0-15 in lane l and rows 16-31 in lane l+32, each stored as one
  // 16-byte write into the column-major byte matrix Wz (row length ldw).
  auto store_block = [&](int8_t* Wz, int tx, int ty, uint32_t R0, uint32_t R1, uint32_t R2,
                         uint32_t R3) {
    const auto s02 = __builtin_amdgcn_permlane32_swap(R0, R2, false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(R1, R3, false, false);
    const int x = xb + tx * 32 + 16 * (lane >> 5);
    const int y = yb + ty * 32 + (lane & 31);
    uint4 v;
    v.x = s02[0];
    v.y = s02[1];
    v.z = s13[0];
    v.w = s13[1];
    *reinterpret_cast<uint4*>(Wz + (size_t)y * ldw + x) = v;
  };
  // Epilogue (EPI 0: mod p_z into W_z; EPI 1: maxima; EPI 2: FP32 store;
  // EPI 3: maxima and nonzero bytes; EPI 4: INT32 store).
  auto finish = [&]() {
    if constexpr (EPI == 4) {
      // INT32 accumulators of slice z stored column-major: D_z[y][x]
      int* Dz = reinterpret_cast<int*>(W) + (size_t)(sidx * nz + z) * sw;
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int x = xb + tx * 32 + 8 * r4 + 4 * (lane >> 5);
            const int y = yb + ty * 32 + (lane & 31);
            *reinterpret_cast<int4*>(Dz + (size_t)y * ldw + x) =
                make_int4(acc[tx][ty][4 * r4 + 0], acc[tx][ty][4 * r4 + 1],
                          acc[tx][ty][4 * r4 + 2], acc[tx][ty][4 * r4 + 3]);
          }
    }
    if constexpr (EPI == 2) {
      // FP32 accumulators stored column-major: S[y][x], 4 consecutive x per lane
      float* S = reinterpret_cast<float*>(W);
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty)
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int x = xb + tx * 32 + 8 * r4 + 4 * (lane >> 5);
            const int y = yb + ty * 32 + (lane & 31);
            *reinterpret_cast<float4*>(S + (size_t)y * ldw + x) =
                make_float4((float)acc[tx][ty][4 * r4 + 0], (float)acc[tx][ty][4 * r4 + 1],
                            (float)acc[tx][ty][4 * r4 + 2], (float)acc[tx][ty][4 * r4 + 3]);
          }
    } else if constexpr (EPI == 0) {
      const int p = cc.p[z];
      int8_t* Wz = W + (size_t)(sidx * nz + z) * sw;
      // The modulus is uniform: one branch for the whole tile.
      if (p == 256) {
#pragma unroll
        for (int tx = 0; tx < TX; ++tx)
#pragma unroll
          for (int ty = 0; ty < TY; ++ty) {
            uint32_t R[4];
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
              R[r4] = pack_bytes(acc[tx][ty][4 * r4 + 0], acc[tx][ty][4 * r4 + 1],
                                 acc[tx][ty][4 * r4 + 2], acc[tx][ty][4 * r4 + 3]);
            store_block(Wz, tx, ty, R[0], R[1], R[2], R[3]);
          }
      } else {
        const double pd = (double)p, pinv = cc.pinv[z];
#pragma unroll
        for (int tx = 0; tx < TX; ++tx)
#pragma unroll
          for (int ty = 0; ty < TY; ++ty) {
            uint32_t R[4];
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
              R[r4] = pack_bytes(mod_odd(acc[tx][ty][4 * r4 + 0], pd, pinv),
                                 mod_odd(acc[tx][ty][4 * r4 + 1], pd, pinv),
                                 mod_odd(acc[tx][ty][4 * r4 + 2], pd, pinv),
                                 mod_odd(acc[tx][ty][4 * r4 + 3], pd, pinv));
            store_block(Wz, tx, ty, R[0], R[1], R[2], R[3]);
          }
      }
    } else if constexpr (EPI == 1 || EPI == 3) {
      if constexpr (EPI == 3) {
#pragma unroll
        for (int tx = 0; tx < TX; ++tx)
#pragma unroll
          for (int ty = 0; ty < TY; ++ty) {
            uint32_t R[4];
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
              R[r4] = pack_bytes(acc[tx][ty][4 * r4 + 0] != 0, acc[tx][ty][4 * r4 + 1] != 0,
                                 acc[tx][ty][4 * r4 + 2] != 0, acc[tx][ty][4 * r4 + 3] != 0);
            store_block(W, tx, ty, R[0], R[1], R[2], R[3]);
          }
      }
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
    }  };

  // k_pad is a multiple of 128.  Group gi lives in half gi % 2 of the LDS; it
  // is issued while group gi-1 is consumed and waited for (all copies done +
  // barrier) before use, which also certifies that every wave has finished
  // reading group gi-1.  No branch encloses an MFMA, so the accumulators stay
  // in place across iterations.
  const int NGall = k_pad / 128;
  const int g_lo = SPLIT ? (int)((int64_t)sidx * NGall / nsplit) : 0;
  const int NG = SPLIT ? (int)((int64_t)(sidx + 1) * NGall / nsplit) : NGall;   // end of this workgroup's groups
  // Within each 32-k sub-step the fragment reads of the next sub-step (into
  // the other register set) alternate one for one with the MFMAs of the
  // current one; the remaining MFMAs follow.
  auto interleave = [&]() {
#pragma unroll
    for (int q = 0; q < TX + TY; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
    }
    if constexpr (TX * TY > TX + TY) __builtin_amdgcn_sched_group_barrier(0x008, TX * TY - (TX + TY), 0);
  };
  // Beyond 2^17 of k (residue products, EPI 0 and its INT32 dump EPI 4) the
  // accumulators are reduced mod p_z (odd p) after every 2^17 of k: a chunk
  // adds at most 127^2 2^17 < 2^31 - 127 in magnitude to a reduced value, so
  // every partial sum stays exact in INT32 and the result is congruent to
  // C'_l mod p_z.  For p = 256 the two's-complement wrap is already exact
  // mod 256.  The inner loop is the same for every chunk.  FOLD selects the
  // build of the kernel for k_pad > 2^17, so that the usual one keeps the
  // plain loop and its register budget.
  constexpr bool kFold = FOLD && (EPI == 0 || EPI == 4);
  const int chunk = kFold ? kFoldGroups : NG - g_lo;
  auto fold = [&]() {
    const int p = cc.p[z];
    if (p == 256) return;
    const double pd = (double)p, pinv = cc.pinv[z];
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[tx][ty][r] = mod_odd(acc[tx][ty][r], pd, pinv);
  };
  issue_x(lds + (SPLIT ? (g_lo & 1) * GROUP_BYTES : 0), z, g_lo * 128);
  issue_y(lds + (SPLIT ? (g_lo & 1) * GROUP_BYTES : 0), z, g_lo * 128);
  for (int g0 = g_lo; g0 < NG; g0 += chunk) {
  const int g1 = min(NG, g0 + chunk);
  for (int gi = g0; gi < g1; ++gi) {
    int8_t* const buf = lds + (gi & 1) * GROUP_BYTES;
    int8_t* const next = lds + ((gi + 1) & 1) * GROUP_BYTES;
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    v4i a0[TX], b0[TY], a1[TX], b1[TY];
    // The first fragment reads go out before the next group's copies, so
    // their LDS latency overlaps the copy issue; the X-row copies follow
    // them and the Y-row copies come one sub-step later, spreading the
    // copies over the first half of the group.
    load_frags(buf, 0, a0, b0);
    if (gi + 1 < NG) issue_x(next, z, (gi + 1) * 128);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(buf, 1, a1, b1);
    mfmas(a0, b0);
    interleave();
    __builtin_amdgcn_sched_barrier(0);
    if (gi + 1 < NG) issue_y(next, z, (gi + 1) * 128);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(buf, 2, a0, b0);
    mfmas(a1, b1);
    interleave();
    __builtin_amdgcn_sched_barrier(0);
    load_frags(buf, 3, a1, b1);
    mfmas(a0, b0);
    interleave();
    __builtin_amdgcn_sched_barrier(0);
    mfmas(a1, b1);
  }
  if constexpr (kFold) {
    if (g1 < NG) fold();
  }
  }
  finish();
}

// Persistent form of the residue products (EPI 0) for batches: a grid of
// resident workgroups walks the block map in a fixed stride (workgroup g
// takes entries g, g + G, g + 2G, ...; G a multiple of 8, so every entry
// runs on the XCD its local index maps to, as in the one-workgroup-per-entry
// launch).  While a workgroup consumes the last k-group of one tile it
// already copies the first k-group of its next tile into the other LDS
// buffer, so that copy overlaps the last MFMAs and the epilogue instead of
// starting the next tile cold; short-k problems spend most of their time in
// that first copy.  The arithmetic of every tile is the one of gemm_body
// (the same fragment order, MFMAs and epilogue), so the results are the same
// bits.
template <int BX, int BY, int NWX, int NWY, bool FOLD>
__device__ __forceinline__ void gemm_persist(const ProbDesc* __restrict__ P,
                                             const BlockRef* __restrict__ map, int items,
                                             const CrtConsts* __restrict__ ctab) {
  constexpr int BK = 128;
  constexpr int NW = NWX * NWY;
  constexpr int WX = BX / NWX, WY = BY / NWY;
  constexpr int TX = WX / 32, TY = WY / 32;
  constexpr int CPR = BK / 16;
  constexpr int RPI = 1024 / BK;
  constexpr int IX = BX / RPI / NW, IY = BY / RPI / NW;
  static_assert(IX % 2 == 0 && IY % 2 == 0 && WX % 32 == 0 && WY % 32 == 0, "tile / wave shape");
  static_assert(BX == BY, "square tiles");
  constexpr int GROUP_BYTES = (BX + BY) * BK;
  constexpr int GROUP = 8;
  __shared__ __attribute__((aligned(1024))) int8_t lds[2 * GROUP_BYTES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wx = wave / NWY, wy = wave % NWY;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int lr = lane / CPR, slot = lane % CPR;
  const int ch_e = (slot ^ swz(lr)) * 16, ch_o = (slot ^ swz(RPI + lr)) * 16;
  const int frow = lane & 31;
  int fo[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) fo[j] = frow * BK + (((2 * j + (lane >> 5)) ^ swz(frow)) * 16);

  // One tile of one residue product.
  struct Job {
    const int8_t* xs;   // this lane's first copy source row of X (slice z, k = 0)
    const int8_t* ys;
    int8_t* Wz;
    int k_pad, ldw, x0, y0, z, p;
    double pinv;
  };
  // Entry i of the map as a job; false for the padding entries.
  auto decode = [&](int i, Job& j) -> bool {
    const BlockRef e = map[i];
    const ProbDesc& d = P[e.x];
    const int tiles_x = d.mp / BX, tiles_y = d.np / BY, nz = d.N;
    const int launched = group_gemm_blocks(d.mp, d.np, BX, nz);
    const int total = tiles_x * tiles_y * nz;
    int bid = e.y;
    {
      const int xcd = bid % kXcds, loc = bid / kXcds;
      const int per = launched / kXcds, extra = launched % kXcds;
      bid = xcd * per + min(xcd, extra) + loc;
    }
    if (bid >= total) return false;
    const int per_slice = tiles_x * tiles_y;
    const int z = bid / per_slice;
    int t = bid % per_slice;
    const int group_span = GROUP * tiles_y;
    const int g = t / group_span;
    const int gx0 = g * GROUP;
    const int gsz = min(GROUP, tiles_x - gx0);
    t -= g * group_span;
    j.x0 = (gx0 + t % gsz) * BX;
    j.y0 = (t / gsz) * BY;
    j.z = z;
    j.k_pad = d.kp;
    j.ldw = d.mp;
    j.xs = d.As + (size_t)z * d.mp * d.kp + (size_t)(j.x0 + wave * IX * RPI + lr) * d.kp;
    j.ys = d.Bs + (size_t)z * d.np * d.kp + (size_t)(j.y0 + wave * IY * RPI + lr) * d.kp;
    j.Wz = d.W + (size_t)z * d.np * d.mp;
    j.p = ctab[d.N].p[z];
    j.pinv = ctab[d.N].pinv[z];
    return true;
  };
  auto issue_x = [&](int8_t* buf, const Job& j, int k0) {
    const uint32_t b = lds_addr(buf);
    const size_t rowstep = (size_t)RPI * j.k_pad;
#pragma unroll
    for (int q = 0; q < IX; ++q)
      dma16(j.xs + k0 + q * rowstep + ((q & 1) ? ch_o : ch_e),
            b + (uint32_t)((wave_u * IX + q) * 1024));
  };
  auto issue_y = [&](int8_t* buf, const Job& j, int k0) {
    const uint32_t b = lds_addr(buf);
    const size_t rowstep = (size_t)RPI * j.k_pad;
#pragma unroll
    for (int q = 0; q < IY; ++q)
      dma16(j.ys + k0 + q * rowstep + ((q & 1) ? ch_o : ch_e),
            b + (uint32_t)(BX * BK + (wave_u * IY + q) * 1024));
  };
  auto next_job = [&](int i, Job& j) -> int {   // first valid entry at or after i (stride G)
    for (; i < items; i += (int)gridDim.x)
      if (decode(i, j)) return i;
    return items;
  };

  v16i acc[TX][TY];
  auto load_frags = [&](const int8_t* buf, int j, v4i (&a)[TX], v4i (&b)[TY]) {
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
      a[tx] = *reinterpret_cast<const v4i*>(buf + (wx * WX + tx * 32) * BK + fo[j]);
#pragma unroll
    for (int ty = 0; ty < TY; ++ty)
      b[ty] = *reinterpret_cast<const v4i*>(buf + (BX + wy * WY + ty * 32) * BK + fo[j]);
  };
  auto mfmas = [&](const v4i (&a)[TX], const v4i (&b)[TY]) {
#pragma unroll
    for (int tx = 0; tx < TX; ++tx)
#pragma unroll
      for (int ty = 0; ty < TY; ++ty)
        acc[tx][ty] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[tx], b[ty], acc[tx][ty], 0, 0, 0);
  };
  auto interleave = [&]() {
#pragma unroll
    for (int q = 0; q < TX + TY; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    if constexpr (TX * TY > TX + TY) __builtin_amdgcn_sched_group_barrier(0x008, TX * TY - (TX + TY), 0);
  };

  Job cur, nxt;
  int i = next_job((int)blockIdx.x, cur);
  if (i >= items) return;   // whole workgroup, before any barrier
  issue_x(lds, cur, 0);
  issue_y(lds, cur, 0);
  int ph = 0;               // LDS buffer of the current job's group 0
  for (;;) {
    const int inext = next_job(i + (int)gridDim.x, nxt);
    const bool more = inext < items;
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
      for (int b = 0; b < TY; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
    const int NG = cur.k_pad / 128;
    for (int g0 = 0; g0 < NG; g0 += FOLD ? kFoldGroups : NG) {
      const int g1 = FOLD ? min(NG, g0 + kFoldGroups) : NG;
      for (int gi = g0; gi < g1; ++gi) {
        int8_t* const buf = lds + ((ph + gi) & 1) * GROUP_BYTES;
        int8_t* const next = lds + ((ph + gi + 1) & 1) * GROUP_BYTES;
        wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        v4i a0[TX], b0[TY], a1[TX], b1[TY];
        load_frags(buf, 0, a0, b0);
        if (gi + 1 < NG)
          issue_x(next, cur, (gi + 1) * 128);
        else if (more)
          issue_x(next, nxt, 0);
        __builtin_amdgcn_sched_barrier(0);
        load_frags(buf, 1, a1, b1);
        mfmas(a0, b0);
        interleave();
        __builtin_amdgcn_sched_barrier(0);
        if (gi + 1 < NG)
          issue_y(next, cur, (gi + 1) * 128);
        else if (more)
          issue_y(next, nxt, 0);
        __builtin_amdgcn_sched_barrier(0);
        load_frags(buf, 2, a0, b0);
        mfmas(a1, b1);
        interleave();
        __builtin_amdgcn_sched_barrier(0);
        load_frags(buf, 3, a1, b1);
        mfmas(a0, b0);
        interleave();
        __builtin_amdgcn_sched_barrier(0);
        mfmas(a1, b1);
      }
      if (FOLD && g1 < NG && cur.p != 256) {   // reduction every 2^17 of k (see gemm_body)
        const double pd = (double)cur.p;
#pragma unroll
        for (int tx = 0; tx < TX; ++tx)
#pragma unroll
          for (int ty = 0; ty < TY; ++ty)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[tx][ty][r] = mod_odd(acc[tx][ty][r], pd, cur.pinv);
      }
    }
    ph = (ph + NG) & 1;
    // epilogue: W_z = mod(C'_z, p_z), as in gemm_body
    const int xb = cur.x0 + wx * WX, yb = cur.y0 + wy * WY;
    auto store_block = [&](int tx, int ty, uint32_t R0, uint32_t R1, uint32_t R2, uint32_t R3) {
      const auto s02 = __builtin_amdgcn_permlane32_swap(R0, R2, false, false);
      const auto s13 = __builtin_amdgcn_permlane32_swap(R1, R3, false, false);
      const int x = xb + tx * 32 + 16 * (lane >> 5);
      const int y = yb + ty * 32 + (lane & 31);
      uint4 v;
      v.x = s02[0];
      v.y = s02[1];
      v.z = s13[0];
      v.w = s13[1];
      *reinterpret_cast<uint4*>(cur.Wz + (size_t)y * cur.ldw + x) = v;
    };
    if (cur.p == 256) {
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty) {
          uint32_t R[4];
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4)
            R[r4] = pack_bytes(acc[tx][ty][4 * r4 + 0], acc[tx][ty][4 * r4 + 1],
                               acc[tx][ty][4 * r4 + 2], acc[tx][ty][4 * r4 + 3]);
          store_block(tx, ty, R[0], R[1], R[2], R[3]);
        }
    } else {
      const double pd = (double)cur.p, pinv = cur.pinv;
#pragma unroll
      for (int tx = 0; tx < TX; ++tx)
#pragma unroll
        for (int ty = 0; ty < TY; ++ty) {
          uint32_t R[4];
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4)
            R[r4] = pack_bytes(mod_odd(acc[tx][ty][4 * r4 + 0], pd, pinv),
                               mod_odd(acc[tx][ty][4 * r4 + 1], pd, pinv),
                               mod_odd(acc[tx][ty][4 * r4 + 2], pd, pinv),
                               mod_odd(acc[tx][ty][4 * r4 + 3], pd, pinv));
          store_block(tx, ty, R[0], R[1], R[2], R[3]);
        }
    }
    if (!more) break;
    cur = nxt;
    i = inext;
  }
}

// Wave grid and residency of the two tile sizes.
template <int B>
struct TileShape;
template <>
struct TileShape<256> {
  static constexpr int NWX = 4, NWY = 2, OCC = 1;
};
template <>
struct TileShape<128> {
  static constexpr int NWX = 2, NWY = 2, OCC = 2;
};
template <int B>
constexpr int tile_threads() {
  return 64 * TileShape<B>::NWX * TileShape<B>::NWY;
}

template <int B, int EPI, bool BF16 = false, bool FOLD = false, bool SPLIT = false>
__global__ __launch_bounds__(tile_threads<B>(), TileShape<B>::OCC) void k_gemm_i8(
    const int8_t* __restrict__ X, size_t sx, const int8_t* __restrict__ Y, size_t sy, int tiles_x,
    int tiles_y, int nz, int k_pad, CrtConsts cc, int8_t* __restrict__ W, size_t sw, int ldw,
    int* __restrict__ xmax, int* __restrict__ ymax, int nsplit) {
  gemm_body<B, B, TileShape<B>::NWX, TileShape<B>::NWY, EPI, BF16, FOLD, SPLIT>(
      X, sx, Y, sy, tiles_x, tiles_y, nz, k_pad, cc, W, sw, ldw, xmax, ymax, blockIdx.x, gridDim.x,
      nsplit);
}

// ---- split-k reductions ------------------------------------------------------
// W (EPI 0): slice z = mod(sum over s of partial slice s * nz + z, p_z); each
// partial is in [-128, 127], so for nsplit <= 64 the sum stays below 2^13 in
// magnitude.  Workgroup row blockIdx.y is slice z; 16 bytes a thread.
__global__ __launch_bounds__(256) void k_reduce_w(const int8_t* __restrict__ part, int nsplit,
                                                  int nz, int64_t sw16, CrtConsts cc,
                                                  int8_t* __restrict__ W) {
  const int z = blockIdx.y;
  const SmallMod md(cc, z);
  const uint4* src = reinterpret_cast<const uint4*>(part);
  uint4* dst = reinterpret_cast<uint4*>(W) + z * sw16;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < sw16;
       t += (int64_t)gridDim.x * 256) {
    int acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0;
    for (int sidx = 0; sidx < nsplit; ++sidx) {
      const uint4 v = src[((int64_t)sidx * nz + z) * sw16 + t];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] += sbyte(w[e >> 2], e & 3);
    }
    uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 16; ++e) o[e >> 2] |= md.byte(acc[e], e & 3);
    dst[t] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

// Cbar (EPI 1) from nsplit INT32 partial sums (column-major, ld nx): one
// entry (x, y) per thread, workgroups of 64 x by 4 y.  Each wave (64
// consecutive x of one y) sends its maximum to ymax[y]; the four rows of a
// workgroup are combined in LDS and sent to xmax[x] (atomicMax, order-free;
// Cbar >= 0).  nx is a multiple of 128.
__global__ __launch_bounds__(256) void k_reduce_cbar(const int* __restrict__ part, int nsplit,
                                                     int nx, int ny, int* __restrict__ xmax,
                                                     int* __restrict__ ymax) {
  __shared__ int rows[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x = blockIdx.x * 64 + tx, y = blockIdx.y * 4 + ty;
  const size_t per = (size_t)nx * ny;
  int v = 0;
  if (y < ny) {
    const int* src = part + (size_t)y * nx + x;
    for (int sidx = 0; sidx < nsplit; ++sidx) v += src[sidx * per];
    int cm = v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cm = max(cm, __shfl_xor(cm, off));
    if (tx == 0) atomicMax(&ymax[y], cm);
  }
  rows[ty][tx] = v;
  __syncthreads();
  if (ty == 0)
    atomicMax(&xmax[x], max(max(rows[0][tx], rows[1][tx]), max(rows[2][tx], rows[3][tx])));
}

// Grouped: the scaling product (EPI 1) or the N residue products (EPI 0) of
// every problem of a batch.
template <int B, int EPI, bool FOLD>
__global__ __launch_bounds__(tile_threads<B>(), TileShape<B>::OCC) void kg_gemm(
    const ProbDesc* __restrict__ P, const BlockRef* __restrict__ map,
    const CrtConsts* __restrict__ ctab) {
  const BlockRef e = map[blockIdx.x];
  const ProbDesc& d = P[e.x];
  const int nz = EPI == 0 ? d.N : 1;
  gemm_body<B, B, TileShape<B>::NWX, TileShape<B>::NWY, EPI, false, FOLD>(
      d.As, EPI == 0 ? (size_t)d.mp * d.kp : 0, d.Bs, EPI == 0 ? (size_t)d.np * d.kp : 0, d.mp / B,
      d.np / B, nz, d.kp, ctab[d.N], d.W, (size_t)d.np * d.mp, d.mp, d.rmax, d.cmax, e.y,
      group_gemm_blocks(d.mp, d.np, B, nz));
}

// Persistent grouped residue products (see gemm_persist).
template <int B, bool FOLD>
__global__ __launch_bounds__(tile_threads<B>(), TileShape<B>::OCC) void kp_gemm(
    const ProbDesc* __restrict__ P, const BlockRef* __restrict__ map, int items,
    const CrtConsts* __restrict__ ctab) {
  gemm_persist<B, B, TileShape<B>::NWX, TileShape<B>::NWY, FOLD>(P, map, items, ctab);
}

template <int B>
void launch_cfg(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                size_t sw, int ldw, int* xmax, int* ymax, int nsplit, bool fold) {
  const int tiles_x = nx_pad / B, tiles_y = ny_pad / B;
  const dim3 grid((unsigned)(tiles_x * tiles_y * nz * nsplit)), block(tile_threads<B>());
#define OZ2_GEMM(E, F, S)                                                                       \
  hipLaunchKernelGGL((k_gemm_i8<B, E, false, F, S>), grid, block, 0, s, X, sx, Y, sy, tiles_x,   \
                     tiles_y, nz, k_pad, cc, W, sw, ldw, xmax, ymax, nsplit)
  const bool split = nsplit > 1;
  switch (epi) {
    case 0:
      if (split) {
        if (fold)
          OZ2_GEMM(0, true, true);
        else
          OZ2_GEMM(0, false, true);
      } else {
        if (fold)
          OZ2_GEMM(0, true, false);
        else
          OZ2_GEMM(0, false, false);
      }
      break;
    case 1:
      OZ2_GEMM(1, false, false);
      break;
    case 3:
      OZ2_GEMM(3, false, false);
      break;
    default:
      if (split)
        OZ2_GEMM(4, false, true);   // the split scaling product (never folded)
      else if (fold)
        OZ2_GEMM(4, true, false);
      else
        OZ2_GEMM(4, false, false);
      break;
  }
#undef OZ2_GEMM
}

// Tile configuration: 0 = automatic; 1 = 256x256, 2 = 128x128 (g_gemm_tile,
// a tuning knob set through ozaki2_debug_tuning).
int forced_cfg() { return g_gemm_tile.load(std::memory_order_relaxed); }

// 256x256 tiles (one workgroup per CU, 128 KB of LDS) when there are more
// than 128 of them, that is when the 128x128 tiles (two workgroups per CU,
// 64 KB of LDS each) would need more than one round of the 512 workgroup
// slots; otherwise 128x128.  Measured on square products from 1024^3 to
// 4096^3 (16 to 896 tiles of 256x256): 144 or more tiles ran 7-25% faster
// as 256x256, 64 or fewer 30-40% faster as 128x128.
bool use_256(int nx_pad, int ny_pad, int nz) {
  const bool fits256 = nx_pad % 256 == 0 && ny_pad % 256 == 0;
  const int cfg = forced_cfg();
  if (cfg == 1 || cfg == 2) return cfg == 1 && fits256;
  const long t256 = (long)(nx_pad / 256) * (ny_pad / 256) * nz;
  return fits256 && t256 > 128;
}

// Split-k of a product with few output workgroups (EPI 0 and 1): with W0 =
// tiles * nz workgroups and G = k_pad / 128 groups of k, nsplit = the number
// of copies of W0 that fill the workgroup slots once (CUs x occupancy: 256
// for 256x256 tiles, 512 for 128x128), at most G / gmin and smax; 1 when W0
// already fills a quarter of the slots.  The residue products take gmin = 4
// (512 k or more per split), smax = 64; the scaling product, whose partials
// are INT32 and which is one product against N, gmin = 32 and smax = 16.
// Measured (FP64, N = 14): 512^2 x 32768 (224 residue workgroups) ran 3%
// slower with two splits than with none; at 1024^2 x 1024 and x 4096 a
// scaling product split 2 and 8 ways was slower than unsplit; at
// 256^2 x 131072 the split products ran 2.4x faster.  A fixed count of 256
// CUs keeps the choice, and with it the workspace size, a function of the
// shape alone.
struct SplitRule {
  int gmin, smax;
};
constexpr SplitRule kSplitRes{4, 64}, kSplitCbar{32, 16};
int choose_split(int nx_pad, int ny_pad, int k_pad, int nz, SplitRule r) {
  if (g_split_k.load(std::memory_order_relaxed) == 1) return 1;
  const int B = use_256(nx_pad, ny_pad, nz) ? 256 : 128;
  const long w0 = (long)(nx_pad / B) * (ny_pad / B) * nz;
  const long slots = B == 256 ? 256 : 512;
  if (w0 <= 0 || 4 * w0 > slots) return 1;
  long sp = slots / w0;
  sp = std::min<long>(sp, (k_pad / 128) / r.gmin);
  sp = std::min<long>(sp, r.smax);
  return sp >= 2 ? (int)sp : 1;
}

}  // namespace

std::atomic<int> g_split_k{0};

size_t split_scratch_bytes(int nx_pad, int ny_pad, int k_pad, int nz) {
  const size_t plane = (size_t)nx_pad * ny_pad;
  const int s0 = choose_split(nx_pad, ny_pad, k_pad, nz, kSplitRes);
  const int s1 = choose_split(nx_pad, ny_pad, k_pad, 1, kSplitCbar);
  const size_t b0 = s0 > 1 ? (size_t)s0 * nz * plane : 0;
  const size_t b1 = s1 > 1 ? (size_t)s1 * plane * 4 : 0;
  return b0 > b1 ? b0 : b1;
}

std::atomic<int> g_gemm_tile{0};

int persist_grid(int tile) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const void* k = tile == 256 ? reinterpret_cast<const void*>(kp_gemm<256, true>)
                              : reinterpret_cast<const void*>(kp_gemm<128, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, tile == 256 ? tile_threads<256>()
                                                                        : tile_threads<128>(),
                                                   0) != hipSuccess ||
      occ < 1)
    occ = 1;
  return (cus * occ + 7) / 8 * 8;   // a multiple of 8: entries keep their XCD
}

void launch_group_gemm_persist(hipStream_t s, int tile, bool fold, int grid, const ProbDesc* P,
                               const BlockRef* map, int items, const CrtConsts* ctab) {
  if (items <= 0) return;
  const dim3 g((unsigned)(grid < items ? grid : (items + 7) / 8 * 8));
  if (tile == 256) {
    const dim3 b(tile_threads<256>());
    if (fold)
      hipLaunchKernelGGL((kp_gemm<256, true>), g, b, 0, s, P, map, items, ctab);
    else
      hipLaunchKernelGGL((kp_gemm<256, false>), g, b, 0, s, P, map, items, ctab);
  } else {
    const dim3 b(tile_threads<128>());
    if (fold)
      hipLaunchKernelGGL((kp_gemm<128, true>), g, b, 0, s, P, map, items, ctab);
    else
      hipLaunchKernelGGL((kp_gemm<128, false>), g, b, 0, s, P, map, items, ctab);
  }
}

void launch_group_gemm(hipStream_t s, int epi, int tile, const ProbDesc* P, const BlockRef* map,
                       int blocks, const CrtConsts* ctab) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks);
  if (tile == 256) {
    const dim3 b(tile_threads<256>());
    if (epi == 0)
      hipLaunchKernelGGL((kg_gemm<256, 0, true>), g, b, 0, s, P, map, ctab);
    else
      hipLaunchKernelGGL((kg_gemm<256, 1, false>), g, b, 0, s, P, map, ctab);
  } else {
    const dim3 b(tile_threads<128>());
    if (epi == 0)
      hipLaunchKernelGGL((kg_gemm<128, 0, true>), g, b, 0, s, P, map, ctab);
    else
      hipLaunchKernelGGL((kg_gemm<128, 1, false>), g, b, 0, s, P, map, ctab);
  }
}

void launch_gemm_bf16_store(hipStream_t s, const uint16_t* X, const uint16_t* Y, int nx_pad,
                            int ny_pad, int k_pad, float* S, int lds_) {
  // BF16 rows are 2*k_pad bytes; the kernel works in bytes of k.
  const int kb = 2 * k_pad;
  CrtConsts cc{};
  if (use_256(nx_pad, ny_pad, 1)) {
    const int tiles_x = nx_pad / 256, tiles_y = ny_pad / 256;
    hipLaunchKernelGGL((k_gemm_i8<256, 2, true>), dim3((unsigned)(tiles_x * tiles_y)),
                       dim3(tile_threads<256>()), 0, s, (const int8_t*)X, 0, (const int8_t*)Y, 0,
                       tiles_x, tiles_y, 1, kb, cc, (int8_t*)S, 0, lds_, nullptr, nullptr, 1);
  } else {
    const int tiles_x = nx_pad / 128, tiles_y = ny_pad / 128;
    hipLaunchKernelGGL((k_gemm_i8<128, 2, true>), dim3((unsigned)(tiles_x * tiles_y)),
                       dim3(tile_threads<128>()), 0, s, (const int8_t*)X, 0, (const int8_t*)Y, 0,
                       tiles_x, tiles_y, 1, kb, cc, (int8_t*)S, 0, lds_, nullptr, nullptr, 1);
  }
}

void launch_gemm_i8(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                    int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                    size_t sw, int ldw, int* xmax, int* ymax, int8_t* part, size_t part_bytes) {
  const bool b256 = use_256(nx_pad, ny_pad, nz);
  const int G = k_pad / 128;
  int sp = 1;
  if (epi == 0 || epi == 1) {
    sp = epi == 0 ? choose_split(nx_pad, ny_pad, k_pad, nz, kSplitRes)
                  : choose_split(nx_pad, ny_pad, k_pad, 1, kSplitCbar);
    const size_t plane = (size_t)nx_pad * ny_pad;
    const size_t need = epi == 0 ? (size_t)sp * nz * plane : (size_t)sp * plane * 4;
    // the partials use the plane layout (stride nx_pad * ny_pad, rows of
    // nx_pad): W must have it too
    const bool plane_w = epi == 1 || (sw == plane && ldw == nx_pad);
    if (sp > 1 && (!part || part_bytes < need || !plane_w)) sp = 1;
  }
  // every split keeps at least one group; fold when a split spans more than 2^17 of k
  const bool fold = (G + sp - 1) / sp > kFoldGroups;
  auto launch = [&](int e, int8_t* out, size_t so, int ld, int* xm, int* ym, int z, bool f) {
    if (b256)
      launch_cfg<256>(s, e, X, sx, Y, sy, nx_pad, ny_pad, k_pad, z, cc, out, so, ld, xm, ym, sp, f);
    else
      launch_cfg<128>(s, e, X, sx, Y, sy, nx_pad, ny_pad, k_pad, z, cc, out, so, ld, xm, ym, sp, f);
  };
  if (sp == 1) {
    launch(epi, W, sw, ldw, xmax, ymax, nz, fold && (epi == 0 || epi == 4));
    return;
  }
  const size_t plane = (size_t)nx_pad * ny_pad;
  if (epi == 0) {
    // partial W of every split (mod p of its partial sum), then their sum mod p
    launch(0, part, plane, nx_pad, nullptr, nullptr, nz, fold);
    const int64_t sw16 = (int64_t)(plane / 16);
    const int64_t b = (sw16 + 255) / 256;
    hipLaunchKernelGGL(k_reduce_w, dim3((unsigned)(b < 1024 ? b : 1024), (unsigned)nz), dim3(256),
                       0, s, part, sp, nz, sw16, cc, W);
  } else {
    // INT32 partial sums of Cbar (never reduced mod p: Cbar < 2^31), then
    // their sum and its row and column maxima
    launch(4, part, plane, nx_pad, nullptr, nullptr, 1, false);
    const dim3 g((unsigned)(nx_pad / 64), (unsigned)((ny_pad + 3) / 4));
    hipLaunchKernelGGL(k_reduce_cbar, g, dim3(256), 0, s, (const int*)part, sp, nx_pad, ny_pad,
                       xmax, ymax);
  }
}

}  // namespace oz2
