// Required number of moduli from the Theorem 1 bound (eq. thm:err-2).
//
// With alpha_i = floor(log2 max_h |a_ih|), beta_j likewise, and the row and
// column powers of two factored out of every quantity, the N-dependent part of
// the bound relative to S_ij = (|A||B|)_ij 2^-(alpha_i + beta_j) is
//   T_ij(N) = t(N) (rs_i sc_j + sr_i cs_j) + (k t(N)^2 + extra(N)) sr_i sc_j,
// where rs_i = sum_h |a_ih| 2^-alpha_i, cs_j likewise for B, sr_i =
// sqrt(max_h Cbar_ih) (2^(e'_i/2)), sc_j likewise, t(N) = 1/sqrt(2^5 (P-1)) and
// extra(N) t^-2 is r_b(N) minus its N-independent output-rounding part.
// rs, cs, sr, sc are rounded up and S_ij is replaced by a lower bound, so every
// decision errs towards a larger N.  Entries with S_ij = 0 are exact zeros and
// are skipped, unless the byte nz_ij (Cbar_ij != 0, which holds exactly when
// (|A||B|)_ij > 0) says the lower bound merely underflowed: such an entry
// accepts no N (and certifies no eps).
#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {
namespace {

// Upward factors: FP64 sums of fewer than 2^19 nonnegative terms are within
// 2^-34 (relative) of the exact sum; one correctly rounded sqrt within 2^-53.
constexpr double kSumUp = 1.0 + 0x1p-30;
constexpr double kSqrtUp = 1.0 + 0x1p-50;
constexpr double kTUp = 1.0 + 0x1p-40;   // a few roundings in T itself

// One workgroup per 64 entries (rows of A first, then columns of B); its four
// waves sum every fourth tile of the partial sums, coalesced across the 64
// entries, and the four partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_plan_vectors(const double* __restrict__ pr, int m_pad,
                                                      const double* __restrict__ pc, int n_pad,
                                                      int tiles, const int* __restrict__ rmax,
                                                      const int* __restrict__ cmax, int m, int n,
                                                      double* __restrict__ rs, double* __restrict__ cs,
                                                      double* __restrict__ sr,
                                                      double* __restrict__ sc) {
  __shared__ double part[4][64];
  const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + e;
  const bool valid = t < m + n;
  const bool row = t < m;
  const int idx = row ? t : t - m;
  double s = 0.0;
  if (valid) {
    const double* p = row ? pr + idx : pc + idx;
    const int stride = row ? m_pad : n_pad;
    for (int q = g; q < tiles; q += 4) s += p[(size_t)q * stride];
  }
  part[g][e] = s;
  __syncthreads();
  if (g != 0 || !valid) return;
  s = (part[0][e] + part[1][e]) + (part[2][e] + part[3][e]);
  const double M = (double)(row ? rmax[idx] : cmax[idx]);
  if (row) {
    rs[idx] = s * kSumUp;
    sr[idx] = sqrt(M) * kSqrtUp;
  } else {
    cs[idx] = s * kSumUp;
    sc[idx] = sqrt(M) * kSqrtUp;
  }
}

__device__ inline bool plan_ok(const PlanTable& pt, int N, double A1, double P2, double target) {
  const double T = (pt.t[N] * A1 + (pt.k * pt.tt[N] + pt.extra[N]) * P2) * kTUp;
  return T <= target;
}

// The per-entry kernels below walk the m x n entries in a grid-stride loop
// over tasks of 256 consecutive i of one column j, and combine their results
// with one atomic per workgroup: one per 256 entries would serialise on the
// single result word (about 11 ns each).
constexpr int kEntryWorkgroups = 2048;

template <typename F>
__device__ __forceinline__ void for_entries(int m, int n, int iblocks, F&& f) {
  const int64_t tasks = (int64_t)iblocks * n;
  for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
    const int j = (int)(task / iblocks);
    const int i = (int)(task % iblocks) * 256 + (int)threadIdx.x;
    if (i < m) f(i, j);
  }
}

// Maximum of v over the workgroup (256 threads), valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_max(T v) {
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
  __shared__ T red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return max(max(red[0], red[1]), max(red[2], red[3]));
}

// Pass 1: a lower bound of the smallest N in [nlo, nhi] that satisfies
// T(N) <= eps S on every entry with S > 0 (nhi + 1 if an entry has none); the
// maximum over the workgroups goes to *out.  Each wave keeps a running bound
// `need` and, for its next 64 entries, looks for the first N >= need that
// each entry satisfies.  Any N that satisfies every entry is >= every such
// first N (by induction over the entries: it is >= each earlier bound, so it
// is one of the candidates searched), so the maximum stays a lower bound;
// pass 2 then searches upward from it.  Most entries pass at the running
// bound in one step.  N advances in step across the wave, so the per-N
// coefficients are wave-uniform (scalar) loads.
__global__ __launch_bounds__(256) void k_plan_entries(const float* __restrict__ S,
                                                      const uint8_t* __restrict__ nz, int lds_,
                                                      int m, int n, int iblocks,
                                                      const double* __restrict__ rs,
                                                      const double* __restrict__ cs,
                                                      const double* __restrict__ sr,
                                                      const double* __restrict__ sc, PlanTable pt,
                                                      int* __restrict__ out) {
  int need = 0;   // wave-uniform running bound
  const int64_t tasks = (int64_t)iblocks * n;
  for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
    const int j = (int)(task / iblocks);
    const int i = (int)(task % iblocks) * 256 + (int)threadIdx.x;
    bool live = false;
    double A1 = 0.0, P2 = 0.0, target = 0.0;
    if (i < m) {
      const double Sl = (double)S[(size_t)j * lds_ + i] * pt.acc_scale;
      if (Sl > 0.0) {
        A1 = rs[i] * sc[j] + sr[i] * cs[j];
        P2 = sr[i] * sc[j];
        target = pt.eps * Sl;
        live = true;
      } else if (nz[(size_t)j * lds_ + i]) {
        live = true;          // nonzero (|A||B|)_ij with no positive lower bound:
        target = -1.0;        // T >= 0 never meets it, so no N is accepted
      }
    }
    int first = 0;
    for (int N = max(pt.nlo, need); N <= pt.nhi; ++N) {
      if (!__any(live)) break;
      if (live && plan_ok(pt, N, A1, P2, target)) {
        first = N;
        live = false;
      }
    }
    if (live) first = pt.nhi + 1;
    for (int off = 32; off >= 1; off >>= 1) first = max(first, __shfl_xor(first, off));
    need = __builtin_amdgcn_readfirstlane(max(need, first));
  }
  need = block_max(need);
  if (threadIdx.x == 0 && need > 0) atomicMax(out, need);
}

// Pass 2: does N satisfy every entry?  Any failure sets *bad.  With Nsrc,
// N is read from there (pass 1's result, at least nlo), and nothing is
// checked if it exceeds nhi.
__global__ __launch_bounds__(256) void k_plan_verify(const float* __restrict__ S,
                                                     const uint8_t* __restrict__ nz, int lds_, int m,
                                                     int n, int iblocks,
                                                     const double* __restrict__ rs,
                                                     const double* __restrict__ cs,
                                                     const double* __restrict__ sr,
                                                     const double* __restrict__ sc, PlanTable pt,
                                                     int N, const int* __restrict__ Nsrc,
                                                     int* __restrict__ bad) {
  if (Nsrc) N = max(__builtin_amdgcn_readfirstlane(*Nsrc), pt.nlo);
  if (N > pt.nhi) return;   // uniform: before any barrier
  int fail = 0;
  for_entries(m, n, iblocks, [&](int i, int j) {
    const double Sl = (double)S[(size_t)j * lds_ + i] * pt.acc_scale;
    if (Sl > 0.0) {
      const double A1 = rs[i] * sc[j] + sr[i] * cs[j];
      const double P2 = sr[i] * sc[j];
      if (!plan_ok(pt, N, A1, P2, pt.eps * Sl)) fail = 1;
    } else if (nz[(size_t)j * lds_ + i]) {
      fail = 1;
    }
  });
  fail = block_max(fail);
  if (threadIdx.x == 0 && fail) atomicOr(bad, 1);
}

// A-posteriori est1 of Theorem 1 (eq. thm:err-1) relative to the lower bound
// of S, per entry.  |A'B'| is bounded through Lemma 4 by the computed C'':
// |A'B'| <= (|C''| + R_const) / (1 - R_rel).  C'' is recovered from the output
// and the shifts: C = C'' 2^-(mu_i + nu_j) rounded once, exactly unless C is
// subnormal, so |C''| <= (|C| + tiny) 2^(mu_i + nu_j) in every case (for b = 32
// this is the FP32 C'' of Algorithm 3, to which Lemma 4 refers).  In factored
// form (row and column powers of two removed, as in the planner):
//   est1 = t A1 + (k t^2 + R_const t^2 + rel (|C''| + R_const)) P2,
// every rounding pushed upward.  The maximum of est1 / S over entries with
// S > 0 goes to *out as the bit pattern of a nonnegative double (whose order
// is that of the unsigned integers).
template <typename T>
__global__ __launch_bounds__(256) void k_certify(const T* __restrict__ C, int ldc,
                                                 const int* __restrict__ mu,
                                                 const int* __restrict__ nu,
                                                 const float* __restrict__ S,
                                                 const uint8_t* __restrict__ nz, int lds_, int m,
                                                 int n, int iblocks, const double* __restrict__ rs,
                                                 const double* __restrict__ cs,
                                                 const double* __restrict__ sr,
                                                 const double* __restrict__ sc, CertTable ct,
                                                 unsigned long long* __restrict__ out) {
  double ratio = 0.0;
  for_entries(m, n, iblocks, [&](int i, int j) {
    const double Sl = (double)S[(size_t)j * lds_ + i] * ct.acc_scale;
    if (Sl > 0.0) {
      const double c = fabs((double)C[i + (size_t)j * ldc]) + ct.tiny;
      const double cpp = ldexp(c, mu[i] + nu[j]);
      const double A1 = rs[i] * sc[j] + sr[i] * cs[j];
      const double P2 = sr[i] * sc[j];
      const double est =
          (ct.t * A1 + (ct.k * ct.tt + ct.extra + ct.rel * (cpp + ct.rconst) * kTUp) * P2) * kTUp;
      ratio = fmax(ratio, est / Sl * kTUp);
    } else if (nz[(size_t)j * lds_ + i]) {
      ratio = INFINITY;     // nonzero (|A||B|)_ij with no positive lower bound
    }
  });
  ratio = block_max(ratio);
  if (threadIdx.x == 0 && ratio > 0.0)
    atomicMax(out, (unsigned long long)__double_as_longlong(ratio));
}

unsigned entry_grid(int iblocks, int n) {
  const int64_t tasks = (int64_t)iblocks * n;
  return (unsigned)(tasks < kEntryWorkgroups ? tasks : kEntryWorkgroups);
}

}  // namespace

void launch_certify(hipStream_t s, Prec pr, const void* C, int ldc, const int* mu, const int* nu,
                    const float* S, const uint8_t* nz, int lds_, int m, int n, const double* rs,
                    const double* cs, const double* sr, const double* sc, const CertTable& ct,
                    unsigned long long* out) {
  const int iblocks = (m + 255) / 256;
  const dim3 grid(entry_grid(iblocks, n)), block(256);
  if (pr == Prec::F64)
    hipLaunchKernelGGL(k_certify<double>, grid, block, 0, s, (const double*)C, ldc, mu, nu, S, nz,
                       lds_, m, n, iblocks, rs, cs, sr, sc, ct, out);
  else
    hipLaunchKernelGGL(k_certify<float>, grid, block, 0, s, (const float*)C, ldc, mu, nu, S, nz,
                       lds_, m, n, iblocks, rs, cs, sr, sc, ct, out);
}

void launch_plan_vectors(hipStream_t s, const double* pr, int m_pad, const double* pc, int n_pad,
                         int tiles, const int* rmax, const int* cmax, int m, int n, double* rs,
                         double* cs, double* sr, double* sc) {
  hipLaunchKernelGGL(k_plan_vectors, dim3((m + n + 63) / 64), dim3(256), 0, s, pr, m_pad, pc,
                     n_pad, tiles, rmax, cmax, m, n, rs, cs, sr, sc);
}

void launch_plan_entries(hipStream_t s, const float* S, const uint8_t* nz, int lds_, int m, int n,
                         const double* rs, const double* cs, const double* sr, const double* sc,
                         const PlanTable& pt, int* out) {
  const int iblocks = (m + 255) / 256;
  hipLaunchKernelGGL(k_plan_entries, dim3(entry_grid(iblocks, n)), dim3(256), 0, s, S, nz,
                     lds_, m, n, iblocks, rs, cs, sr, sc, pt, out);
}

void launch_plan_verify(hipStream_t s, const float* S, const uint8_t* nz, int lds_, int m, int n,
                        const double* rs, const double* cs, const double* sr, const double* sc,
                        const PlanTable& pt, int N, const int* Nsrc, int* bad) {
  const int iblocks = (m + 255) / 256;
  hipLaunchKernelGGL(k_plan_verify, dim3(entry_grid(iblocks, n)), dim3(256), 0, s, S, nz,
                     lds_, m, n, iblocks, rs, cs, sr, sc, pt, N, Nsrc, bad);
}

}  // namespace oz2
