// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace oz2 {

constexpr int kMaxModuli = 49;   // Section 3.1: p_l <= 256 pairwise coprime => N <= 49
constexpr int kMaxK = 1 << 17;   // Section 3: k <= 2^17
constexpr int kRowPad = 256;     // m and n are padded to this multiple in the workspace
constexpr int kKPad = 128;       // k is padded to this multiple (bytes of INT8 per row)

// Per-(N, b) constants of Section 3.1 and Algorithms 2-3, passed to kernels
// by value (they land in the kernel-argument segment and are read with
// scalar loads).
struct CrtConsts {
  int N;
  int b;            // 64 or 32
  int nsteps;       // exact-reduction steps for |A'| < 2^(6 + floor(P'))
  float Pprime;     // P' = single_down(log2(P-1)/2 - 0.5)
  float c;          // single_down(-0.5 / (1 - 4 u_32))
  double P1, P2;    // double-double P (P2 = 0 for b = 32)
  double Pinv;      // double(1/P)
  int p[kMaxModuli];
  double pinv[kMaxModuli];  // double(1/p_l)
  double s1[kMaxModuli];    // s_l1
  double s2[kMaxModuli];    // s_l2 (0 for b = 32)
};

// Host-side tables (tables.cpp).  Returns false if a constant could not be
// established (e.g. P' too close to the FP32 grid for the host's precision).
bool build_consts(int N, int b, CrtConsts* out);
// N-dependent coefficients of the planner bound for every N in [2, 49]:
//   t(N) = 1/sqrt(32 (P-1)), tt(N) = t^2, extra(N) = (r_b(N) - r_rnd) t^2,
//   rnd(N) = r_rnd t^2 (the N-independent output rounding part).
struct PlanCoef {
  double t[kMaxModuli + 1];
  double tt[kMaxModuli + 1];
  double extra[kMaxModuli + 1];
  double rnd[kMaxModuli + 1];
};
bool build_plan_coef(int b, PlanCoef* out);

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
// Kernel launchers (each defined next to its kernel)
// ---------------------------------------------------------------------------
enum class Prec { F64, F32 };

// scale.hip
void launch_init(hipStream_t s, uint64_t* rowbits, int m_pad, uint64_t* colbits, int n_pad,
                 int* rmax, int* cmax, int* flag);
void launch_absmax_rows(hipStream_t s, Prec pr, const void* A, int lda, int m, int k,
                        uint64_t* rowbits, int* flag);
void launch_absmax_cols(hipStream_t s, Prec pr, const void* B, int ldb, int k, int n,
                        uint64_t* colbits, int* flag);
void launch_shifts(hipStream_t s, const uint64_t* rowbits, const int* rmax, int m,
                   const uint64_t* colbits, const int* cmax, int n, float Pprime, float c,
                   int* mu_p, int* nu_p, int* mu, int* nu, float* ef);
void launch_log2f(hipStream_t s, const float* d, float* out, int count);

// residue.hip: INT8 slices in K-major layout [S][rows_pad][k_pad].
//   src element (r, h) is at  trans ? src[r + h*ld] : src[h + r*ld].
//   mode 0 (bar):     S = 1, byte = ceil(2^shift |x|) (>= 1 if x != 0),
//                     shift = mu' computed from `bits` (row abs-max bit patterns)
//   mode 1 (residue): S = N, byte_l = mod(trunc(2^shift x), p_l), shift from `shift`
void launch_slices(hipStream_t s, Prec pr, int mode, bool trans, const void* src, int ld, int rows,
                   int k, int rows_pad, int k_pad, const uint64_t* bits, const int* shift,
                   const CrtConsts& cc, int8_t* out);

// gemm_i8.hip
//   D[x][y] = sum_h X[x][h] * Y[y][h] over k_pad, for slices z = 0..nz-1 with
//   X_z = X + z*sx, Y_z = Y + z*sy (X: A side, x = i; Y: B side, y = j).
//   epi 0: W_z[y][x] = mod(D, p_z) as int8 into W + z*sw, row length ldw.
//   epi 1: xmax[x] = max_y D, ymax[y] = max_x D (atomicMax; D >= 0).
void launch_gemm_i8(hipStream_t s, int epi, const int8_t* X, size_t sx, const int8_t* Y, size_t sy,
                    int nx_pad, int ny_pad, int k_pad, int nz, const CrtConsts& cc, int8_t* W,
                    size_t sw, int ldw, int* xmax, int* ymax);

// crt.hip: C(i, j) from W_l[j][i] (slices of row length ldw), mu, nu.
void launch_crt(hipStream_t s, Prec pr, const int8_t* W, size_t sw, int ldw, const int* mu,
                const int* nu, int m, int n, const CrtConsts& cc, const int* flag, void* C,
                int ldc);
void launch_fill_zero(hipStream_t s, Prec pr, void* C, int ldc, int m, int n);
// Folds the per-call non-finite flag into the sticky status word.
void launch_or_status(hipStream_t s, const int* flag, int* status);

}  // namespace oz2
