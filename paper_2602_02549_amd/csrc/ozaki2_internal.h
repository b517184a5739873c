// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>

namespace oz2 {

constexpr int kMaxModuli = 49;   // Section 3.1: p_l <= 256 pairwise coprime => N <= 49
// k < 2^19: Section 3 assumes k <= 2^17; beyond it Cbar <= 2^12 k stays below
// 2^31 and the residue products are reduced mod p_l every 2^17 of k.
constexpr int kMaxK = (1 << 19) - 1;
constexpr int kRowPad = 256;     // m and n are padded to this multiple in the workspace
constexpr int kMaxDim = 0x7FFFFF00; // largest m, n whose padding to kRowPad fits in int
constexpr int kKPad = 128;       // k is padded to this multiple (bytes of INT8 per row)
constexpr int kCrtRows = 4;      // CRT: consecutive rows per thread (256 threads per block)

// Per-(N, b) constants of Section 3.1 and Algorithms 2-3, passed to kernels
// by value (they land in the kernel-argument segment and are read with
// scalar loads).
struct CrtConsts {
  int N;
  int b;            // 64 or 32
  int table;        // moduli: kTablePaper or kTableOptimal
  int nsteps;       // exact-reduction steps for |A'| < 2^(6 + floor(P'))
  int nlimbs;       // 2 or 3: residues from limbs of A' (0: use nsteps)
  float Pprime;     // P' = single_down(log2(P-1)/2 - 0.5)
  float c;          // single_down(-0.5 / (1 - 4 u_32))
  double P1, P2;    // double-double P (P2 = 0 for b = 32)
  double Pinv;      // double(1/P)
  int p[kMaxModuli];
  double pinv[kMaxModuli];  // double(1/p_l)
  double s1[kMaxModuli];    // s_l1
  double s2[kMaxModuli];    // s_l2 (0 for b = 32)
};

// Moduli tables (Section 3.1): the first N of the paper's fixed list, or the
// N pairwise coprime integers <= 256 of largest product (descending).
constexpr int kTablePaper = 0;
constexpr int kTableOptimal = 1;
bool moduli_of(int table, int N, int* p);

// Host-side tables (tables.cpp).  Returns false if a constant could not be
// established (e.g. P' too close to the FP32 grid for the host's precision).
bool build_consts(int N, int b, int table, CrtConsts* out);
// N-dependent coefficients of the planner bound for every N in [2, 49]:
//   t(N) = 1/sqrt(32 (P-1)), tt(N) = t^2, extra(N) = (r_b(N) - r_rnd) t^2,
//   rnd(N) = r_rnd t^2 (the N-independent output rounding part).
struct PlanCoef {
  double t[kMaxModuli + 1];
  double tt[kMaxModuli + 1];
  double extra[kMaxModuli + 1];
  double rnd[kMaxModuli + 1];
  double rconst[kMaxModuli + 1];  // R_const of Lemma 4
  double rel[kMaxModuli + 1];     // R_rel t^2 / (1 - R_rel)
};
bool build_plan_coef(int b, int table, PlanCoef* out);

// The a-posteriori est1 of Theorem 1 at one N, in the planner's factored form
// (passed by value to the certification kernel).
struct CertTable {
  double t, tt, extra;  // t(N), t(N)^2, R_const t(N)^2
  double rconst, rel;   // R_const; R_rel t(N)^2 / (1 - R_rel)
  double k;             // inner dimension
  double acc_scale;     // lower-bound factor of the BF16 product S
  double tiny;          // smallest positive subnormal of the output type
};

// Everything the per-entry planner kernels need (passed by value).
struct PlanTable {
  int nlo, nhi;        // search range of N
  double k;            // inner dimension
  double eps;          // target
  double acc_scale;    // lower-bound factor for the FP32-accumulated BF16 product
  double t[kMaxModuli + 1], tt[kMaxModuli + 1], extra[kMaxModuli + 1];
};

// mu' = 5 - floor(log2 x) (Algorithm 2, eq. mu'nu') from the IEEE bit pattern
// of x = max_h |a_ih| as an FP64 number; a zero row gets 0 (its outputs are
// exact zeros).  Exact for subnormals.
__device__ inline int shift_prime_bits(uint64_t bits) {
  if (bits == 0) return 0;
  int ex = (int)(bits >> 52);
  if (ex == 0x7FF) return 0;  // non-finite input: every output is forced to NaN
  int fl;
  if (ex == 0) {
    uint64_t mant = bits & 0x000FFFFFFFFFFFFFull;
    fl = (63 - __clzll((long long)mant)) - 1074;
  } else {
    fl = ex - 1023;
  }
  return 5 - fl;
}

// ---------------------------------------------------------------------------
// Grouped (batched) execution: one launch per phase covers every problem of a
// batch.  Each problem has a descriptor; per phase, a block map gives every
// workgroup its problem and its index among that problem's workgroups (one
// uniform load, no search).
struct ProbDesc {
  int m, n, k, N;
  int mp, np, kp;           // padded sizes (workspace layout)
  int lda, ldb, ldc;
  const void* A;
  const void* B;
  void* C;
  uint64_t* rowbits;
  uint64_t* colbits;
  int* rmax;
  int* cmax;
  int* mu;
  int* nu;
  int* flag;
  int8_t* As;               // [N][mp][kp]
  int8_t* Bs;               // [N][np][kp]
  int8_t* W;                // [N][np][mp]
};

// Block map entry: x = problem index, y = local workgroup index.
typedef int2 BlockRef;

enum GroupPhase {
  GP_INIT, GP_ABSMAX_A, GP_ABSMAX_B, GP_ABSBAR_B, GP_SLICE_A, GP_SLICE_B, GP_GEMM_SCALE, GP_SHIFTS,
  GP_GEMM_RES, GP_CRT, GP_COUNT
};

__host__ __device__ inline int cdiv_i(int a, int b) { return (a + b - 1) / b; }

// Workgroups of one problem in the grouped init phase (a grid-stride loop over
// max(mp, np) entries) and in a grouped product with `tile` x `tile` output
// tiles and nz slices (padded to a multiple of 8 so that every problem starts
// on XCD 0).
__host__ __device__ inline int group_init_blocks(int mp, int np) {
  return cdiv_i(mp > np ? mp : np, 256);
}
__host__ __device__ inline int group_gemm_blocks(int mp, int np, int tile, int nz) {
  return ((mp / tile) * (np / tile) * nz + 7) / 8 * 8;
}
// Workgroups of the CRT (one thread per kCrtRows rows of one column) and of
// the column abs-max (one wave per column, four per workgroup).
__host__ __device__ inline int64_t crt_blocks(int m, int n) {
  return ((int64_t)cdiv_i(m, kCrtRows) * n + 255) / 256;
}
__host__ __device__ inline int absmax_cols_blocks(int n) { return cdiv_i(n, 4); }

// ---------------------------------------------------------------------------
// Kernel launchers (each defined next to its kernel)
// ---------------------------------------------------------------------------
enum class Prec { F64, F32 };

// scale.hip
void launch_init(hipStream_t s, uint64_t* rowbits, int m_pad, uint64_t* colbits, int n_pad,
                 int* rmax, int* cmax, int* flag);
// cx: the matrix holds interleaved (re, im) pairs (leading dimension in
// complex elements) and each maximum runs over both parts.  dup > 0: row i's
// maximum also goes to row i + dup.
void launch_absmax_rows(hipStream_t s, Prec pr, const void* A, int lda, int m, int k,
                        uint64_t* rowbits, int* flag, bool cx = false, int dup = 0);
void launch_absmax_cols(hipStream_t s, Prec pr, const void* B, int ldb, int k, int n,
                        uint64_t* colbits, int* flag, bool cx = false);
// Abs-max of the columns of B and Bbar (slice 0, K-major [n_pad][k_pad]) in
// one read of B; for k_pad <= kAbsBarMaxK.
constexpr int kAbsBarMaxK = 8192;
constexpr int kAbsBarWaveK = 2048;   // up to here one wave per column, else a workgroup
int absbar_group_blocks(int n_pad, int k_pad);
void launch_absbar_cols(hipStream_t s, Prec pr, const void* B, int ldb, int k, int n, int n_pad,
                        int k_pad, uint64_t* colbits, int* flag, int8_t* out);
// bias: added to mu' and nu' of nonzero rows and columns (0 for Algorithm 2;
// -1 for the complex 3-product form, whose bars sum two parts).
void launch_shifts(hipStream_t s, const uint64_t* rowbits, const int* rmax, int m,
                   const uint64_t* colbits, const int* cmax, int n, float Pprime, float c,
                   int* mu_p, int* nu_p, int* mu, int* nu, float* ef, int bias = 0);
void launch_log2f(hipStream_t s, const float* d, float* out, int count);

// Tuning and test knobs (ozaki2_debug_tuning): a cap on the workgroups of a
// slice launch (0: none; residue.hip) and the forced tile of the single-problem
// products (0: automatic, 1: 256x256, 2: 128x128; gemm_i8.hip).
extern std::atomic<int> g_slice_cap;
extern std::atomic<int> g_gemm_tile;
// Split-k of the single-problem products: 0 automatic (default), 1 off.
extern std::atomic<int> g_split_k;

// residue.hip: per-device launch figures of the slice kernels (resident workgroups);
// called once per device before its first launch, outside stream capture.
void init_slice_launch(int dev);

// residue.hip: INT8 slices in K-major layout [S][rows_pad][k_pad].
//   src element (r, h) is at  trans ? src[r + h*ld] : src[h + r*ld].
//   mode 0 (bar):     S = 1, byte = ceil(2^shift |x|) (>= 1 if x != 0),
//                     shift = mu' computed from `bits` (row abs-max bit patterns)
//   mode 2 (bar):     mode 0 with shift = mu' - 1 (the complex 3-product form)
//   mode 1 (residue): S = N, byte_l = mod(trunc(2^shift x), p_l), shift from `shift`
void launch_slices(hipStream_t s, Prec pr, int mode, bool trans, const void* src, int ld, int rows,
                   int k, int rows_pad, int k_pad, const uint64_t* bits, const int* shift,
                   const CrtConsts& cc, int8_t* out);
// The same passes over an interleaved complex source (the 3-product form),
// each reading the complex matrix once:
//   mode 2: one slice at out, byte = ceil(2^(mu'-1) |re|) + ceil(2^(mu'-1) |im|);
//   mode 1: 3 N slices from out: the residues of the real parts, of the
//           imaginary parts, and of their sums (mod p_l of the two bytes).
void launch_slices_complex(hipStream_t s, Prec pr, int mode, bool trans, const void* src, int ld,
                           int rows, int k, int rows_pad, int k_pad, const uint64_t* bits,
                           const int* shift, const CrtConsts& cc, int8_t* out);
// The slices of the real embedding Ahat = [[Ar, -Ai], [Ai, Ar]],
// Bhat = [[Br], [Bi]] of a complex product, read from the interleaved
// complex source in place (modes 0 and 1 as launch_slices).  The embedding
// is laid out with its halves at aligned offsets, zeros between: k-half kh
// (a multiple of 128; slice rows are 2 kh long) and, on the A side, row half
// `half` (rows i and half + i of the embedding come from complex row i;
// rows_pad = 2 half).  Zero rows and columns change none of the embedding's
// products, maxima or shifts.  Mode 1 on the A side takes the shifts of row
// i from shift[i] and of row half + i from shift[half + i].
void launch_slices_embed(hipStream_t s, Prec pr, int mode, bool aside, const void* src, int ld,
                         int rows, int k, int kh, int rows_pad, int half, const uint64_t* bits,
                         const int* shift, const CrtConsts& cc, int8_t* out);

// Planner operands (BF16, K-major [rows_pad][k_pad]) and per-64-k-tile row
// sums partial[k_pad/64][rows_pad] of |x| 2^-alpha.
void launch_plan_slices(hipStream_t s, Prec pr, bool trans, const void* src, int ld, int rows,
                        int k, int rows_pad, int k_pad, const uint64_t* bits, uint16_t* out,
                        double* partial);

// gemm_i8.hip
//   D[x][y] = sum_h X[x][h] * Y[y][h] over k_pad, for slices z = 0..nz-1 with
//   X_z = X + z*sx, Y_z = Y + z*sy (X: A side, x = i; Y: B side, y = j).
//   epi 0: W_z[y][x] = mod(D, p_z) as int8 into W + z*sw, row length ldw.
//   epi 1: xmax[x] = max_y D, ymax[y] = max_x D (atomicMax; D >= 0).
//   epi 3: epi 1, and W[y][x] = (D != 0) as one byte (row length ldw).
//   epi 4: D_z[y][x] as INT32 into (int*)W + z*sw, row length ldw (elements).
//   part, part_bytes: scratch for split-k (epi 0 and 1, when few output
//   tiles leave the CUs idle): the partial products of the k ranges go there
//   and a reduction kernel combines them into the same result (epi 0: the
//   sum of the partial mod-p bytes, mod p; epi 1: the INT32 sum, then its
//   maxima).  With too little scratch (or none) the product is not split.
void launch_gemm_i8(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                    int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                    size_t sw, int ldw, int* xmax, int* ymax, int8_t* part = nullptr,
                    size_t part_bytes = 0);
// Scratch bytes that lets launch_gemm_i8 split both the scaling product (epi
// 1) and the nz residue products (epi 0) of this shape; 0 if neither splits.
size_t split_scratch_bytes(int nx_pad, int ny_pad, int k_pad, int nz);

// S[y][x] = sum_h X[x][h] Y[y][h] over BF16 slices (FP32 accumulation on
// the matrix cores), stored column-major with row length lds_.
void launch_gemm_bf16_store(hipStream_t s, const uint16_t* X, const uint16_t* Y, int nx_pad,
                            int ny_pad, int k_pad, float* S, int lds_);

// plan.hip
void launch_plan_vectors(hipStream_t s, const double* pr, int m_pad, const double* pc, int n_pad,
                         int tiles, const int* rmax, const int* cmax, int m, int n, double* rs,
                         double* cs, double* sr, double* sc);
// S: lower bound of (|A||B|)_ij (scaled), nz: one byte per entry, nonzero
// exactly when (|A||B|)_ij > 0; both column-major with row length lds_.
void launch_plan_entries(hipStream_t s, const float* S, const uint8_t* nz, int lds_, int m, int n,
                         const double* rs, const double* cs, const double* sr, const double* sc,
                         const PlanTable& pt, int* out);
// N from Nsrc (device) when it is not null; see k_plan_verify.
void launch_plan_verify(hipStream_t s, const float* S, const uint8_t* nz, int lds_, int m, int n,
                        const double* rs, const double* cs, const double* sr, const double* sc,
                        const PlanTable& pt, int N, const int* Nsrc, int* bad);
// Maximum over entries of the a-posteriori est1 / S (bit pattern into *out,
// which the caller zeroes); C is the output of the run whose shifts are mu, nu.
void launch_certify(hipStream_t s, Prec pr, const void* C, int ldc, const int* mu, const int* nu,
                    const float* S, const uint8_t* nz, int lds_, int m, int n, const double* rs,
                    const double* cs, const double* sr, const double* sc, const CertTable& ct,
                    unsigned long long* out);

// Grouped launches (one per phase for a whole batch of `count` problems);
// `map` holds `blocks` entries, one per workgroup.
void launch_group_scale(hipStream_t s, Prec pr, int phase, const ProbDesc* P, const BlockRef* map,
                        int blocks, const CrtConsts* ctab);
// The residue path every problem of a batch shares (a code for
// launch_group_slices), or the per-tile choice when they differ.
int group_residue_path(const CrtConsts* const* cc, int count);
void launch_group_slices(hipStream_t s, Prec pr, int mode, bool aside, int path,
                         const ProbDesc* P, const BlockRef* map, int blocks,
                         const CrtConsts* ctab);
void launch_group_gemm(hipStream_t s, int epi, int tile, const ProbDesc* P, const BlockRef* map,
                       int blocks, const CrtConsts* ctab);
// Persistent grouped residue products: `grid` resident workgroups (a multiple
// of 8, from persist_grid, queried outside any capture) walk the `items`
// entries of the block map.
int persist_grid(int tile);
// `fold`: some problem has k_pad > 2^17 (the build with reductions mod p).
void launch_group_gemm_persist(hipStream_t s, int tile, bool fold, int grid, const ProbDesc* P,
                               const BlockRef* map, int items, const CrtConsts* ctab);
void launch_group_crt(hipStream_t s, Prec pr, const ProbDesc* P, const BlockRef* map, int blocks,
                      int count, const CrtConsts* ctab, int* status);

// crt.hip: C(i, j) from W_l[j][i] (slices of row length ldw), mu, nu.
void launch_crt(hipStream_t s, Prec pr, const int8_t* W, size_t sw, int ldw, const int* mu,
                const int* nu, int m, int n, const CrtConsts& cc, const int* flag, void* C,
                int ldc);
// The CRT of a complex result: real parts from (Wr, mur), imaginary parts
// from (Wi, mui), column shifts nu, written as interleaved (re, im) pairs into
// the column-major complex C (ldc in complex elements).
void launch_crt_complex(hipStream_t s, Prec pr, const int8_t* Wr, const int8_t* Wi, size_t sw,
                        int ldw, const int* mur, const int* mui, const int* nu, int m, int n,
                        const CrtConsts& cc, const int* flag, void* C, int ldc);
// The CRT of the 3-product form: the real and imaginary residues of modulus l
// are mod(W1 - W2, p_l) and mod(W3 - W1 - W2, p_l), formed per byte from the
// three products' W; shifts mu (rows) and nu (columns) for both parts;
// interleaved complex output as launch_crt_complex.
void launch_crt_3m(hipStream_t s, Prec pr, const int8_t* W1, const int8_t* W2, const int8_t* W3,
                   size_t sw, int ldw, const int* mu, const int* nu, int m, int n,
                   const CrtConsts& cc, const int* flag, void* C, int ldc);
// launch_crt plus C'(1), C'(2), Q, C'' as FP64 [4][n][m] into dbg (stage dumps).
void launch_crt_debug(hipStream_t s, Prec pr, const int8_t* W, size_t sw, int ldw, const int* mu,
                      const int* nu, int m, int n, const CrtConsts& cc, const int* flag, void* C,
                      int ldc, double* dbg);
void launch_fill_zero(hipStream_t s, Prec pr, void* C, int ldc, int m, int n);
// Folds the per-call non-finite flag into the sticky status word.
void launch_or_status(hipStream_t s, const int* flag, int* status);

// complex.hip: the real embedding of a complex product (interleaved (re, im)
// column-major inputs; leading dimensions in complex elements) into
// Ahat = [[Ar, -Ai], [Ai, Ar]] (2m x 2k, ld 2m) and Bhat = [[Br], [Bi]]
// (2k x n, ld 2k).
void launch_embed_complex(hipStream_t s, Prec pr, const void* A, int lda, const void* B, int ldb,
                          int m, int n, int k, void* Ah, void* Bh);

// api.cpp: Algorithm 1 for one problem on a workspace of `cap` bytes that
// `get` supplies, with its sticky status word; checks the arguments and the
// size (OZAKI2_ERR_WORKSPACE if the layout needs more than cap) before any
// HIP call and allocates nothing.
typedef int (*BufferSource)(char** ws, int** status);
int gemm_on_buffer(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                   void* C, int ldc, int N, size_t cap, BufferSource get);
// noalloc.hip: the status word of the allocation-free entry point on device
// `dev`, or nullptr while that entry point has not been set up there.
int* noalloc_status(int dev);

// probe.hip: the MFMA-rate probe (ozaki2_debug_mfma_probe): `blocks`
// workgroups of 8 waves, `iters` steps of 8 MFMAs each, operands changing
// every step or fixed; returns its duration (ms, HIP events on s,
// synchronised) and its INT8 operation count.
int probe_mfma(hipStream_t s, int blocks, int iters, bool change, float* ms, double* ops);

}  // namespace oz2
