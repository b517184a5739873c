/*
 * ozaki2.h - C ABI of the MI355X (gfx950) Ozaki-II emulated GEMM library.
 *
 * The library computes C ~= A*B for FP64 (DGEMM emulation) or FP32 (SGEMM
 * emulation) matrices with the accurate-mode Ozaki-II scheme of
 * Uchino, Ozaki and Imamura, "Error Analysis of Matrix Multiplication
 * Emulation Using Ozaki-II Scheme" (arXiv 2602.02549):
 *   Algorithm 2 (Scaling): per-row / per-column power-of-two shifts mu, nu
 *     chosen from an INT8 product of 6-bit magnitude bounds, then truncation
 *     A' = trunc(diag(2^mu) A), B' = trunc(B diag(2^nu));
 *   Algorithm 3 (CRT): INT8 residues A'_l = mod(A', p_l), B'_l = mod(B', p_l)
 *     for the first N moduli of the fixed list of Section 3.1, N exact
 *     INT8 x INT8 -> INT32 products C'_l = A'_l B'_l on the matrix cores,
 *     W_l = mod(C'_l, p_l), and the double-double CRT reduction to C'';
 *   Algorithm 1: C = diag(2^-mu) C'' diag(2^-nu).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major (BLAS): element (i, j) of an m x n matrix X
 *     with leading dimension ldx is X[i + (size_t)j * ldx].  C := A*B
 *     (alpha = 1, beta = 0).
 *   - Every matrix pointer is a DEVICE pointer on the current HIP device.
 *     The caller owns A, B and C; A and B are only read, C is only written.
 *   - Work is enqueued on the stream set with ozaki2_set_stream (default:
 *     the null stream) and the calls return without waiting for it.
 *     Argument errors are detected on the host before anything is enqueued.
 *   - Errors are negative ozaki2_status values.  Data-dependent conditions
 *     found on the device (non-finite input) are reported by
 *     ozaki2_sync_status.
 *   - The library keeps one workspace per device, grown on demand with
 *     hipMalloc unless the caller installs its own with ozaki2_set_workspace.
 *     Calls that overlap on one device race on that workspace; the library
 *     is meant to be driven from one host thread per device.
 *   - ozaki2_gemm and ozaki2_sgemm enqueue kernels only (no memset or copy):
 *     after one call on the device has set up its state, and with a
 *     workspace already large enough, a call can be captured into a graph
 *     by the caller and replayed.
 */
#ifndef OZAKI2_H
#define OZAKI2_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OZAKI2_OK = 0,
  OZAKI2_ERR_INVALID_ARG = -1, /* m,n,k < 0; m or n > 2^31 - 256; lda < max(1,m);
                                  ldb < max(1,k); ldc < max(1,m); NULL pointer for a matrix
                                  with a nonzero extent                                      */
  OZAKI2_ERR_N_RANGE = -2,     /* N outside [2, 49] (FP64) or [2, 16] (FP32)                  */
  OZAKI2_ERR_K_RANGE = -3,     /* k >= 2^19 (Sections 3-4 assume k <= 2^17; up to 2^19 - 1
                                  the library keeps every step exact, see ozaki2_gemm)        */
  OZAKI2_ERR_WORKSPACE = -4,   /* caller-installed workspace smaller than required            */
  OZAKI2_ERR_UNREACHABLE = -5, /* required_moduli: no admissible N meets eps                  */
  OZAKI2_ERR_NONFINITE = -6,   /* an input entry was Inf or NaN (reported by sync_status)     */
  OZAKI2_ERR_HIP = -7,         /* a HIP runtime call failed                                   */
  OZAKI2_ERR_INIT = -8         /* constant tables could not be built                          */
} ozaki2_status;

/*
 * ozaki2_gemm - FP64 C := A*B by Algorithm 1 with b = 64 and moduli p_1..p_N.
 *   m, n, k : sizes; A is m x k, B is k x n, C is m x n (column-major).
 *   N       : number of moduli, 2 <= N <= 49 (Algorithms 1-3 preconditions).
 * Accuracy: |AB - C| obeys Theorem 1 (eq. thm:err-1) entrywise.
 * k: 0 <= k < 2^19.  The paper assumes k <= 2^17; above it, Cbar = Abar Bbar
 * (at most 2^12 k) still fits INT32 exactly, and each residue product is
 * reduced mod p_l after every 2^17 of k, so W_l = mod(A'_l B'_l, p_l) stays
 * exact and Lemmas 0-4 and Theorem 1 hold as stated (Lemma 1's proof with
 * log2 Cbar < 31 in place of 29).
 * k == 0 writes C = 0; m == 0 or n == 0 does nothing.
 * If an input entry is non-finite every entry of C is set to NaN and
 * ozaki2_sync_status later returns OZAKI2_ERR_NONFINITE.
 * Split-k: when C has too few output tiles to occupy the GPU and k is long,
 * the scaling product and the residue products run over k ranges in
 * parallel; the partial products are combined exactly (mod p_l for the
 * residue products, as INT32 sums for Cbar), so the results are the same
 * bits.  The workspace includes room for the partials.
 * Returns OZAKI2_OK or an argument / HIP error.
 */
int ozaki2_gemm(int m, int n, int k, const double *A, int lda, const double *B, int ldb,
                double *C, int ldc, int N);

/*
 * ozaki2_sgemm - FP32 C := A*B by Algorithm 1 with b = 32 (s_l2 = P2 = 0,
 * C'' rounded to FP32 before the inverse scaling, Algorithm 3 last step).
 *   N : 2 <= N <= 16, so that single(C'') cannot overflow (|A'B'| < P/2 by
 *       Lemma 0 and P/2 < 2^128 up to N = 16).
 * Other arguments and behaviour as ozaki2_gemm.
 */
int ozaki2_sgemm(int m, int n, int k, const float *A, int lda, const float *B, int ldb,
                 float *C, int ldc, int N);

/*
 * ozaki2_zgemm - complex FP64 C := A*B (ZGEMM emulation); ozaki2_cgemm the
 * complex FP32 form (b = 32, N <= 16).  Sections 1.1 and 7 name complex
 * emulation and leave its analysis to future work; here the real method of
 * Algorithm 1 runs unchanged on the real embedding
 *     [[Ar, -Ai], [Ai, Ar]] (2m x 2k)  times  [[Br], [Bi]] (2k x n),
 * whose product holds Re(AB) in its first m rows and Im(AB) in the rest, so
 * Lemmas 0-4 and Theorem 1 bound the error of each real and imaginary part
 * as for a real product with inner dimension 2k (four real residue products
 * of the complex sizes per modulus).  Each row of the embedding gets its own
 * shift: the real and imaginary parts of a row of C are scaled separately.
 *   A, B, C : DEVICE pointers to interleaved (re, im) pairs (C99 complex /
 *             std::complex layout), column-major; lda, ldb, ldc count complex
 *             elements (lda >= max(1,m), ldb >= max(1,k), ldc >= max(1,m),
 *             ldc < 2^30).
 *   k       : 0 <= k < 2^18 (the real limit applies to 2k).
 *   N       : as ozaki2_gemm / ozaki2_sgemm.
 * Workspace: ozaki2_complex_workspace_bytes (library-managed or installed).
 * Returns and reports like ozaki2_gemm.
 */
int ozaki2_zgemm(int m, int n, int k, const double *A, int lda, const double *B, int ldb,
                 double *C, int ldc, int N);
int ozaki2_cgemm(int m, int n, int k, const float *A, int lda, const float *B, int ldb, float *C,
                 int ldc, int N);
/*
 * ozaki2_zgemm3m / ozaki2_cgemm3m - the same products with three real
 * residue products per modulus instead of four (Gauss's identity):
 * T1 = A'r B'r, T2 = A'i B'i, T3 = (A'r + A'i)(B'r + B'i), Re = T1 - T2,
 * Im = T3 - T1 - T2, reduced mod p_l and rebuilt by the CRT of Algorithm 3.
 * The three products share one shift per row of A and per column of B, so
 * Algorithm 2 runs on the complex matrices as wholes: mu' is one lower than
 * the real one and Abar = ceil(2^mu' |Ar|) + ceil(2^mu' |Ai|), so that
 * Lemma 0 bounds (|A'r| + |A'i|)(|B'r| + |B'i|), hence both parts, below P/2.
 * The results differ from ozaki2_zgemm's (other shifts); each part's error
 * is bounded as stated in the library's documentation of this form.
 *   k : 0 <= k < 2^19.  Other arguments as ozaki2_zgemm / ozaki2_cgemm.
 */
int ozaki2_zgemm3m(int m, int n, int k, const double *A, int lda, const double *B, int ldb,
                   double *C, int ldc, int N);
int ozaki2_cgemm3m(int m, int n, int k, const float *A, int lda, const float *B, int ldb,
                   float *C, int ldc, int N);
/* Bytes of device workspace the complex calls (prec 64: ozaki2_zgemm,
 * ozaki2_zgemm3m; prec 32: ozaki2_cgemm, ozaki2_cgemm3m) need: the larger of
 * the two forms (the 3-product form only, for k >= 2^18); 0 for arguments
 * they would reject and for m, n or k == 0. */
size_t ozaki2_complex_workspace_bytes(int prec, int m, int n, int k, int N);

/*
 * ozaki2_required_moduli - smallest N for which the N-dependent part of the
 * Theorem 1 bound (eq. thm:err-2 without the N-independent output rounding)
 * is at most eps times (|A||B|)_ij for every entry (i, j) with a nonzero
 * (|A||B|)_ij.  Section 5 and the conclusion state that the bound tells how
 * many moduli a target accuracy needs; this call applies it.
 *   prec  : 64 (A, B are const double*) or 32 (const float*).
 *   A, B  : device matrices as in ozaki2_gemm / ozaki2_sgemm.
 *   eps   : target (> 0).
 *   N_out : HOST pointer; receives N (or the largest admissible N when the
 *           target is unreachable, with OZAKI2_ERR_UNREACHABLE returned).
 * (|A||B|)_ij is replaced by a certified lower bound, which can only raise N.
 * Synchronises the stream (N is returned to the host).
 */
int ozaki2_required_moduli(int prec, int m, int n, int k, const void *A, int lda, const void *B,
                           int ldb, double eps, int *N_out);
/*
 * ozaki2_zrequired_moduli - the same for the complex product of ozaki2_zgemm
 * (prec 64, complex128 pairs) or ozaki2_cgemm (prec 32): the planner applied
 * to the real embedding [[Ar, -Ai], [Ai, Ar]] x [[Br], [Bi]] on which those
 * calls run, so that every real and imaginary part of C meets the target
 * relative to its entry of |Ahat||Bhat| ((|Ar||Br| + |Ai||Bi|) for the real
 * part, (|Ai||Br| + |Ar||Bi|) for the imaginary part).  Arguments as
 * ozaki2_zgemm (no C); k < 2^18.  The 3-product form has other shifts and is
 * not covered.
 */
int ozaki2_zrequired_moduli(int prec, int m, int n, int k, const void *A, int lda,
                            const void *B, int ldb, double eps, int *N_out);

/*
 * ozaki2_gemm_certified - C := A*B like ozaki2_gemm (prec 64) or ozaki2_sgemm
 * (prec 32), with N chosen so that the whole Theorem 1 bound est1
 * (eq. thm:err-1, output rounding included) is at most eps times
 * (|A||B|)_ij on every entry with a nonzero (|A||B|)_ij, certified after the
 * run: the |A'B'| that est1 contains is bounded through Lemma 4 by the
 * computed C'', |A'B'| <= (|C''| + R_const) / (1 - R_rel).  Starting at
 * N_start (0: the N of ozaki2_required_moduli, never above the certified
 * one), the call runs Algorithm 1, evaluates est1 and, if some entry misses
 * eps, runs again with N + 1.
 *   eps     : target (> 0).  FP64 output rounding alone makes est1 exceed
 *             about 1e-15 (|A||B|)_ij, so targets near 1e-15 are
 *             unreachable; 1e-14 is typical.
 *   N_start : 0, or the first N to try (range as for ozaki2_gemm / sgemm).
 *   N_used  : HOST pointer; receives the N of the C returned.
 *   ratio   : HOST pointer or NULL; receives max_ij est1_ij / S_ij at N_used,
 *             with S_ij a certified lower bound of (|A||B|)_ij (as in
 *             ozaki2_required_moduli), every rounding taken upward.
 * Returns OZAKI2_OK when certified; OZAKI2_ERR_UNREACHABLE when no N up to
 * the maximum (49, or 16 for prec 32) certifies eps (C then holds the result
 * at that N); OZAKI2_ERR_NONFINITE for a non-finite input entry (C is NaN);
 * argument / workspace / HIP errors as ozaki2_gemm.  k == 0 writes C = 0.
 * An output entry that is subnormal keeps only a bound on C'', so such
 * entries can fail to certify.  Synchronises the stream.  The workspace
 * needed is ozaki2_certified_workspace_bytes at the largest N tried.
 */
int ozaki2_gemm_certified(int prec, int m, int n, int k, const void *A, int lda, const void *B,
                          int ldb, void *C, int ldc, double eps, int N_start, int *N_used,
                          double *ratio);

/* Bytes of device workspace ozaki2_gemm_certified needs at N (0 for
 * arguments the call would reject, and for m, n or k == 0). */
size_t ozaki2_certified_workspace_bytes(int prec, int m, int n, int k, int N);

/* Work queue: every later call on this host thread enqueues on `stream`
 * (a hipStream_t; NULL = the null stream). */
int ozaki2_set_stream(void *stream);

/*
 * ozaki2_set_moduli_table - the moduli every later call on this host thread
 * uses (Section 3.1, Determination of Constants):
 *   OZAKI2_MODULI_PAPER   (default) the first N entries of the fixed list of
 *                         49 pairwise coprime moduli <= 256 (eq. p_list);
 *   OZAKI2_MODULI_OPTIMAL for each N, the N pairwise coprime integers in
 *                         [2, 256] of largest product P (Section 3.1 notes
 *                         that this set depends on N -- 255 leaves it from
 *                         N = 7 on -- and can be tabulated per N), in
 *                         descending order.
 * Every constant of Section 3.1 (P, q_l, s_l1, s_l2, P1, P2, P_inv, P') and
 * of the Theorem 1 bounds follows the table.  Returns OZAKI2_OK or
 * OZAKI2_ERR_INVALID_ARG for an unknown table.
 * ozaki2_moduli writes the N moduli of `table` to p_out (HOST array of N
 * ints); OZAKI2_ERR_N_RANGE for N outside [2, 49].
 * ozaki2_debug_constants writes, for parity checks against the CPU oracle,
 * the FP64 values P1, P2, P_inv, P', c, s_1..s_N(1), s_1..s_N(2) of (prec,
 * table, N) to out (HOST array of 5 + 2N doubles).
 */
enum { OZAKI2_MODULI_PAPER = 0, OZAKI2_MODULI_OPTIMAL = 1 };
int ozaki2_set_moduli_table(int table);
int ozaki2_moduli(int table, int N, int *p_out);
int ozaki2_debug_constants(int prec, int table, int N, double *out);

/* Bytes of device workspace a call with these sizes needs (prec 64 or 32);
 * 0 for arguments the call itself would reject. */
size_t ozaki2_workspace_bytes(int prec, int m, int n, int k, int N);

/* Install a caller-owned device workspace for the current device (NULL, 0
 * returns to the library-managed one).  The buffer must stay valid while
 * calls that use it are in flight. */
int ozaki2_set_workspace(void *dptr, size_t bytes);

/*
 * ozaki2_gemm_noalloc - for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): ozaki2_gemm (prec 64) or ozaki2_sgemm (prec 32) with the same
 * arguments, results and asynchrony, but its workspace is a fixed device
 * array of OZAKI2_NOALLOC_SCRATCH_BYTES per device, owned by the library and
 * held from the device's first call until the process ends.  The call
 * allocates nothing: no hipMalloc, no hipFree, no allocating library call,
 * and it ignores any workspace installed with ozaki2_set_workspace.
 *   prec : 64 (A, B, C are double*) or 32 (float*).
 * Returns OZAKI2_ERR_WORKSPACE, before anything is enqueued, when the call
 * needs more than that array holds (ozaki2_workspace_bytes(prec, m, n, k, N)
 * + 256 > OZAKI2_NOALLOC_SCRATCH_BYTES; e.g. FP64 2048^3 fits up to N = 21).
 * Every call on one device shares that device's array, so calls that
 * overlap on one device (other streams, other host threads) race on it.
 * A non-finite input is reported by ozaki2_sync_status as for ozaki2_gemm.
 */
#define OZAKI2_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int ozaki2_gemm_noalloc(int prec, int m, int n, int k, const void *A, int lda, const void *B,
                        int ldb, void *C, int ldc, int N);

/* Wait for the stream, then return OZAKI2_OK or the first data-dependent
 * status recorded since the previous ozaki2_sync_status (and clear it). */
int ozaki2_sync_status(void);

/*
 * ozaki2_gemm_batched - `count` independent emulated GEMMs of uneven sizes
 * and per-problem N, run as one launch per phase of Algorithm 1 over all
 * problems; results are bit-identical to `count` separate calls.
 *   prec            : 64 (double) or 32 (float) for every problem.
 *   mnkN            : HOST array of 4*count ints (m, n, k, N per problem).
 *   A, B, C         : HOST arrays of `count` device pointers.
 *   lda, ldb, ldc   : HOST arrays of `count` leading dimensions.
 * Each problem obeys the rules of ozaki2_gemm / ozaki2_sgemm; any invalid
 * problem makes the whole call fail before anything is enqueued.
 * The first call with a given batch (sizes, N, pointers, leading dimensions
 * and workspace) builds a device problem table, runs the batch once, times
 * the residue products under each tile split and form (one workgroup per
 * tile, persistent workgroups, and, in a batch of at most 64 problems of
 * which some split k, one launch per problem) on the residues that run
 * produced, captures the launch sequence with the fastest into a hipGraph
 * and synchronises the stream; later calls with the same batch replay the graph
 * asynchronously and allocate nothing.  Up to eight batches stay cached per
 * device.  The workspace needed is ozaki2_batched_workspace_bytes.
 */
int ozaki2_gemm_batched(int prec, int count, const int *mnkN, const void *const *A,
                        const int *lda, const void *const *B, const int *ldb, void *const *C,
                        const int *ldc);

/* Bytes of device workspace ozaki2_gemm_batched needs for these problems
 * (mnkN as for ozaki2_gemm_batched); 0 for invalid arguments. */
size_t ozaki2_batched_workspace_bytes(int prec, int count, const int *mnkN);

/*
 * ozaki2_debug_stages - run Algorithms 1-3 like ozaki2_gemm / ozaki2_sgemm
 * and copy the intermediate quantities into caller buffers (device pointers;
 * any may be NULL to skip it).  For parity checks against the CPU oracle.
 *   nout    : number of entries of out (10..16); entries past it count as NULL.
 *   out[0]  int32 [m]          mu'      (Algorithm 2)
 *   out[1]  int32 [n]          nu'
 *   out[2]  int32 [m]          row maxima of Cbar = Abar*Bbar
 *   out[3]  int32 [n]          column maxima of Cbar
 *   out[4]  int32 [m]          mu
 *   out[5]  int32 [n]          nu
 *   out[6]  int8  [N][m][k]    A'_l  (row-major per modulus: k contiguous)
 *   out[7]  int8  [N][n][k]    B'_l^T (k contiguous per column of B)
 *   out[8]  int8  [N][n][m]    W_l   (column-major per modulus)
 *   out[9]  double/float [n][m] C (column-major, ldc = m); required
 *   out[10] float [m+n]        log2f values e (rows) then f (columns)
 *   out[11] int32 [N][n][m]    C'_l = A'_l B'_l as INT32 (Algorithm 3), from
 *                              the residue-product kernel with the tile
 *                              choice of the call (two's-complement wrap);
 *                              for k > 2^17 the accumulator as it ends after
 *                              its reductions mod p_l, congruent to C'_l
 *   out[12] double [n][m]      C'(1) (Algorithm 3 / Lemma 2)
 *   out[13] double [n][m]      C'(2) (0 for prec 32)
 *   out[14] double [n][m]      Q     (Lemma 3)
 *   out[15] double [n][m]      C''   (Lemma 4; the FP32 value for prec 32)
 * Allocates temporary device memory for out[11..15].  Returns like
 * ozaki2_gemm (OZAKI2_ERR_INVALID_ARG also for nout outside 10..16 or a
 * NULL out[9]).  Synchronises the stream.
 */
int ozaki2_debug_stages(int prec, int m, int n, int k, const void *A, int lda, const void *B,
                        int ldb, int N, int nout, void *const *out);

/*
 * ozaki2_debug_log2f - the library's log2f (Algorithm 2; correctly rounded
 * to nearest FP32, which meets the accuracy assumption eq. assumption:log2)
 * applied to `count` FP32 values d[i] >= 1 (device pointers).  For the
 * exhaustive check over all integer-valued FP32 inputs in [1, 2^29].
 */
int ozaki2_debug_log2f(const float *d, float *out, int count);

/*
 * ozaki2_debug_mfma_probe - a measurement aid for the roofline of the residue
 * products: one workgroup of 8 waves per CU issues `iters` steps of 8
 * v_mfma_i32_32x32x32_i8 (the residue products' instruction, 2 x 32^3 INT8
 * operations each), with no memory traffic, on operands that change every
 * step (changing = 1: the rate the chip sustains for that instruction on
 * changing data under its power limit) or stay fixed (changing = 0: the
 * issue rate with little data toggling).  *ms (HOST) receives its duration,
 * *ops (HOST) its operation count.  Synchronises the stream.
 * OZAKI2_ERR_INVALID_ARG for iters outside [1, 2^20] (2^20 steps take about
 * 0.4 s), changing not 0 or 1, or NULL outputs.
 */
int ozaki2_debug_mfma_probe(int iters, int changing, float *ms, double *ops);

/*
 * ozaki2_profile - per-kernel timing with HIP events on the library stream.
 *   enable != 0 turns recording on (and clears previous records); 0 off.
 * ozaki2_profile_read copies up to `cap` records (name index, milliseconds)
 * of the calls made since the last enable; returns the number of records.
 * ozaki2_profile_name returns the kernel-phase name of an index.
 */
int ozaki2_profile(int enable);
int ozaki2_profile_read(int *phase, float *ms, int cap);
const char *ozaki2_profile_name(int phase);

/*
 * ozaki2_debug_tuning - process-wide tuning and test knobs (normal use needs
 * none of them).  Sets knob to value and stores the old value in *previous
 * (HOST pointer, may be NULL).  Affects calls made after it; a batch already
 * captured keeps the choices it was captured with unless its knobs differ.
 *   OZAKI2_KNOB_SLICE_WORKGROUPS : cap on the workgroups of each residue /
 *                                  slice launch (0 = none, the default)
 *   OZAKI2_KNOB_GEMM_TILE        : product tile of single-problem calls
 *                                  (0 = automatic, 1 = 256x256, 2 = 128x128)
 *   OZAKI2_KNOB_BATCH_SPLIT      : batched calls: -1 = autotune (default);
 *                                  s >= 0: problems with at least s output
 *                                  tiles of 256x256 per product use them
 *   OZAKI2_KNOB_BATCH_GRAPH      : 1 = capture a batch into a hipGraph
 *                                  (default), 0 = enqueue its kernels directly
 *   OZAKI2_KNOB_BATCH_PERSIST    : batched residue products: -1 = autotune
 *                                  (default), 0 = one workgroup per tile,
 *                                  1 = persistent workgroups, 2 = one
 *                                  launch per problem for the scaling and
 *                                  residue products, splitting k where a
 *                                  problem's output leaves the GPU idle
 *                                  (split-k scratch is held for batches of
 *                                  at most 64 problems)
 *   OZAKI2_KNOB_SPLIT_K          : single-problem products: 0 = split k
 *                                  when few output tiles would leave the
 *                                  compute units idle (default), 1 = never
 * Returns OZAKI2_OK, or OZAKI2_ERR_INVALID_ARG for an unknown knob or value.
 */
enum {
  OZAKI2_KNOB_SLICE_WORKGROUPS = 0,
  OZAKI2_KNOB_GEMM_TILE = 1,
  OZAKI2_KNOB_BATCH_SPLIT = 2,
  OZAKI2_KNOB_BATCH_GRAPH = 3,
  OZAKI2_KNOB_BATCH_PERSIST = 4,
  OZAKI2_KNOB_SPLIT_K = 5
};
int ozaki2_debug_tuning(int knob, int value, int *previous);

/* Library version string. */
const char *ozaki2_version(void);

#ifdef __cplusplus
}
#endif
#endif /* OZAKI2_H */
