// C ABI of the Ozaki-II emulated GEMM (include/ozaki2.h): argument checks,
// workspace management, constant-table cache and the launch sequence of
// Algorithm 1 (Scaling -> CRT -> inverse scaling) on one HIP stream.
#include "../../include/ozaki2.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "ozaki2_internal.h"

using namespace oz2;

namespace {

thread_local hipStream_t g_stream = nullptr;
thread_local int g_table = kTablePaper;   // moduli table of this host thread's calls

constexpr int kDebugOutputs = 16;   // entries of ozaki2_debug_stages' output list

struct BatchEntry;

struct DeviceState {
  void* ws = nullptr;          // library-owned workspace
  size_t ws_bytes = 0;
  void* user_ws = nullptr;     // caller-installed workspace (takes precedence)
  size_t user_bytes = 0;
  uint64_t ws_gen = 1;         // bumped whenever the workspace address may change
  int* status = nullptr;       // sticky data-dependent status word
  CrtConsts* ctab[2][2] = {};  // device tables of CrtConsts by N: [moduli table][b = 64, 32]
  hipStream_t capture = nullptr;            // library stream used only for graph capture
  std::vector<std::shared_ptr<BatchEntry>> batches;  // captured batches, oldest first
};
std::mutex g_mu;
// Never destroyed: its entries own device resources, and HIP must not be
// called from static destructors at process exit.
std::map<int, DeviceState>& g_dev = *new std::map<int, DeviceState>;
std::map<int, CrtConsts> g_consts;  // key: (table * 100 + N) * 100 + b
PlanCoef g_plan[2][2];              // planner coefficients: [moduli table][b = 64, 32]
bool g_plan_ok[2][2] = {};

// ---------------------------------------------------------------------------
// profiling (HIP events around each phase on the library stream)
// ---------------------------------------------------------------------------
enum Phase {
  PH_INIT, PH_ABSMAX_A, PH_ABSMAX_B, PH_BAR_A, PH_BAR_B, PH_GEMM_SCALE, PH_SHIFTS, PH_RES_A,
  PH_RES_B, PH_GEMM_RES, PH_CRT, PH_PLAN, PH_BATCH, PH_COUNT
};
const char* kPhaseNames[PH_COUNT] = {"init", "absmax_A", "absmax_B", "bar_A", "bar_B",
                                     "gemm_scale", "shifts", "residue_A", "residue_B",
                                     "gemm_residue", "crt", "plan", "batched"};
struct ProfRec {
  int phase;
  hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_recs;

struct Scope {
  ProfRec rec{};
  bool on;
  Scope(int phase, hipStream_t s) : on(g_prof) {
    if (!on) return;
    rec.phase = phase;
    if (hipEventCreate(&rec.a) != hipSuccess || hipEventCreate(&rec.b) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(rec.a, s);
    stream = s;
  }
  ~Scope() {
    if (!on) return;
    (void)hipEventRecord(rec.b, stream);
    g_recs.push_back(rec);
  }
  hipStream_t stream = nullptr;
};

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
size_t rup(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int mp, np, kp;
  size_t rowbits, colbits, rmax, cmax, mu_p, nu_p, mu, nu, ef, flag, A, B, W, part, part_bytes,
      total;
};

// Row padding of one problem's layout.  The products use 256x256 tiles when
// there are more than 128 of them, which needs m and n padded to 256.  Below
// 512 such tiles the padding to 256 is taken only if it adds at most 1/8 to
// the output area of the padding to 128; otherwise 128x128 tiles on the
// smaller padding.
int single_row_pad(int m, int n, int N) {
  const int64_t m1 = m > 0 ? m : 1, n1 = n > 0 ? n : 1;
  const int64_t a256 = (int64_t)rup((size_t)m1, 256) * (int64_t)rup((size_t)n1, 256);
  const int64_t a128 = (int64_t)rup((size_t)m1, 128) * (int64_t)rup((size_t)n1, 128);
  const int64_t t = a256 / (256 * 256) * N;
  if (t >= 512) return 256;
  return (t > 128 && 8 * a256 <= 9 * a128) ? 256 : 128;
}

// In a batch, a problem may use 256x256 tiles only if padding it to 256
// costs at most 1/8 more output area than padding to 128, and it has at
// least 4 such tiles.
int batch_row_pad(int m, int n) {
  const int64_t a256 = (int64_t)rup((size_t)m, 256) * (int64_t)rup((size_t)n, 256);
  const int64_t a128 = (int64_t)rup((size_t)m, 128) * (int64_t)rup((size_t)n, 128);
  return (8 * a256 <= 9 * a128 && a256 >= 4 * 256 * 256) ? 256 : 128;
}

// split_nz > 0: room for the split-k partials of the scaling product and of
// residue-product launches of split_nz slices (single-problem calls).
Layout layout(int m, int n, int k, int N, int pad, int split_nz = 0) {
  Layout L;
  L.mp = (int)rup((size_t)(m > 0 ? m : 1), pad);
  L.np = (int)rup((size_t)(n > 0 ? n : 1), pad);
  L.kp = (int)rup((size_t)(k > 0 ? k : 1), kKPad);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = rup(off + bytes, 256);
    return o;
  };
  L.rowbits = take(8ull * L.mp);
  L.colbits = take(8ull * L.np);
  L.rmax = take(4ull * L.mp);
  L.cmax = take(4ull * L.np);
  L.mu_p = take(4ull * L.mp);
  L.nu_p = take(4ull * L.np);
  L.mu = take(4ull * L.mp);
  L.nu = take(4ull * L.np);
  L.ef = take(4ull * ((size_t)L.mp + L.np));
  L.flag = take(4);
  L.A = take((size_t)N * L.mp * L.kp);
  L.B = take((size_t)N * L.np * L.kp);
  L.W = take((size_t)N * L.np * L.mp);
  L.part_bytes = split_nz > 0 ? split_scratch_bytes(L.mp, L.np, L.kp, split_nz) : 0;
  L.part = take(L.part_bytes);
  L.total = off;
  return L;
}

int check_args(int m, int n, int k, const void* A, int lda, const void* B, int ldb, const void* C,
               int ldc, bool needC) {
  if (m < 0 || n < 0 || k < 0 || m > kMaxDim || n > kMaxDim) return OZAKI2_ERR_INVALID_ARG;
  if (lda < (m > 1 ? m : 1) || ldb < (k > 1 ? k : 1)) return OZAKI2_ERR_INVALID_ARG;
  if (needC && ldc < (m > 1 ? m : 1)) return OZAKI2_ERR_INVALID_ARG;
  if ((size_t)m * k > 0 && !A) return OZAKI2_ERR_INVALID_ARG;
  if ((size_t)k * n > 0 && !B) return OZAKI2_ERR_INVALID_ARG;
  if (needC && (size_t)m * n > 0 && !C) return OZAKI2_ERR_INVALID_ARG;
  if (k > kMaxK) return OZAKI2_ERR_K_RANGE;
  return OZAKI2_OK;
}

int check_N(int N, int b) {
  if (N < 2) return OZAKI2_ERR_N_RANGE;
  if (b == 64 && N > kMaxModuli) return OZAKI2_ERR_N_RANGE;
  if (b == 32 && N > 16) return OZAKI2_ERR_N_RANGE;
  return OZAKI2_OK;
}

// Constants of the calling thread's moduli table.
int get_consts(int N, int b, CrtConsts* out) {
  const int table = g_table;
  std::lock_guard<std::mutex> lk(g_mu);
  int key = (table * 100 + N) * 100 + b;
  auto it = g_consts.find(key);
  if (it == g_consts.end()) {
    CrtConsts cc;
    if (!build_consts(N, b, table, &cc)) return OZAKI2_ERR_INIT;
    it = g_consts.emplace(key, cc).first;
  }
  *out = it->second;
  return OZAKI2_OK;
}

// Returns a device workspace of at least `bytes` for the current device.
int get_workspace(size_t bytes, char** base, int** status, uint64_t* gen = nullptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& st = g_dev[dev];
  if (!st.status) {
    init_slice_launch(dev);
    if (hipMalloc(&st.status, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
    if (hipMemset(st.status, 0, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
  }
  *status = st.status;
  if (st.user_ws) {
    if (st.user_bytes < bytes) return OZAKI2_ERR_WORKSPACE;
    *base = (char*)st.user_ws;
    if (gen) *gen = st.ws_gen;
    return OZAKI2_OK;
  }
  if (st.ws_bytes < bytes) {
    if (st.ws) {
      if (hipDeviceSynchronize() != hipSuccess) return OZAKI2_ERR_HIP;
      (void)hipFree(st.ws);
      st.ws = nullptr;
      st.ws_bytes = 0;
    }
    ++st.ws_gen;
    if (hipMalloc(&st.ws, bytes) != hipSuccess) return OZAKI2_ERR_HIP;
    st.ws_bytes = bytes;
  }
  *base = (char*)st.ws;
  if (gen) *gen = st.ws_gen;
  return OZAKI2_OK;
}

struct PlanLayout {
  int mp, np, kp;
  size_t rowbits, colbits, rmax, cmax, flag, res, Abar, Bbar, Abf, Bbf, pr, pc, rs, cs, sr, sc, S,
      mask, total;
};

PlanLayout plan_layout(int m, int n, int k) {
  PlanLayout L;
  L.mp = (int)rup((size_t)m, kRowPad);
  L.np = (int)rup((size_t)n, kRowPad);
  L.kp = (int)rup((size_t)k, kKPad);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = rup(off + bytes, 256);
    return o;
  };
  const size_t tiles = L.kp / 64;
  L.rowbits = take(8ull * L.mp);
  L.colbits = take(8ull * L.np);
  L.rmax = take(4ull * L.mp);
  L.cmax = take(4ull * L.np);
  L.flag = take(4);
  L.res = take(8);
  L.Abar = take((size_t)L.mp * L.kp);
  L.Bbar = take((size_t)L.np * L.kp);
  L.Abf = take(2ull * L.mp * L.kp);
  L.Bbf = take(2ull * L.np * L.kp);
  L.pr = take(8ull * tiles * L.mp);
  L.pc = take(8ull * tiles * L.np);
  L.rs = take(8ull * L.mp);
  L.cs = take(8ull * L.np);
  L.sr = take(8ull * L.mp);
  L.sc = take(8ull * L.np);
  L.S = take(4ull * L.mp * L.np);
  L.mask = take((size_t)L.mp * L.np);
  L.total = off;
  return L;
}

int get_plan_coef(int b, PlanCoef* out) {
  const int table = g_table;
  std::lock_guard<std::mutex> lk(g_mu);
  const int i = b == 64 ? 0 : 1;
  if (!g_plan_ok[table][i]) {
    if (!build_plan_coef(b, table, &g_plan[table][i])) return OZAKI2_ERR_INIT;
    g_plan_ok[table][i] = true;
  }
  *out = g_plan[table][i];
  return OZAKI2_OK;
}

template <typename P>
P* at(char* base, size_t off) {
  return reinterpret_cast<P*>(base + off);
}

// Results of the scaling pass (Algorithm 2 up to the maxima of Cbar) that a
// caller has already computed for the same A and B: the row and column
// abs-max bit patterns, the maxima of Cbar and the non-finite flag.
struct PreScale {
  const uint64_t* rowbits;
  const uint64_t* colbits;
  const int* rmax;
  const int* cmax;
  int* flag;
};

// The launch sequence of Algorithm 1 for one problem (m, n, k >= 1).  With
// `pre`, the scaling pass is taken from there and not run again.
int run_pipeline(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                 void* C, int ldc, const CrtConsts& cc, const Layout& L, char* ws, int* status,
                 hipStream_t s, bool want_ef, const PreScale* pre = nullptr) {
  uint64_t* rowbits = at<uint64_t>(ws, L.rowbits);
  uint64_t* colbits = at<uint64_t>(ws, L.colbits);
  int* rmax = at<int>(ws, L.rmax);
  int* cmax = at<int>(ws, L.cmax);
  int* flag = at<int>(ws, L.flag);
  int8_t* As = at<int8_t>(ws, L.A);
  int8_t* Bs = at<int8_t>(ws, L.B);
  int8_t* W = at<int8_t>(ws, L.W);
  int* mu = at<int>(ws, L.mu);
  int* nu = at<int>(ws, L.nu);
  if (pre) {
    rowbits = const_cast<uint64_t*>(pre->rowbits);
    colbits = const_cast<uint64_t*>(pre->colbits);
    rmax = const_cast<int*>(pre->rmax);
    cmax = const_cast<int*>(pre->cmax);
    flag = pre->flag;
  } else {
    {
      Scope sc(PH_INIT, s);
      launch_init(s, rowbits, L.mp, colbits, L.np, rmax, cmax, flag);
    }
    {
      Scope sc(PH_ABSMAX_A, s);
      launch_absmax_rows(s, pr, A, lda, m, k, rowbits, flag);
    }
    // Abar = ceil(2^mu' |A|), Bbar = ceil(|B| 2^nu') into slice 0 of the operand buffers.
    // Up to kAbsBarMaxK the abs-max of B and Bbar come from one read of B.
    const bool fuse_b = L.kp <= kAbsBarMaxK;
    if (!fuse_b) {
      Scope sc(PH_ABSMAX_B, s);
      launch_absmax_cols(s, pr, B, ldb, k, n, colbits, flag);
    }
    {
      Scope sc(PH_BAR_A, s);
      launch_slices(s, pr, 0, true, A, lda, m, k, L.mp, L.kp, rowbits, nullptr, cc, As);
    }
    {
      Scope sc(PH_BAR_B, s);
      if (fuse_b)
        launch_absbar_cols(s, pr, B, ldb, k, n, L.np, L.kp, colbits, flag, Bs);
      else
        launch_slices(s, pr, 0, false, B, ldb, n, k, L.np, L.kp, colbits, nullptr, cc, Bs);
    }
    // Cbar = Abar Bbar; keep row maxima (over j) and column maxima (over i).
    {
      Scope sc(PH_GEMM_SCALE, s);
      launch_gemm_i8(s, 1, As, 0, Bs, 0, L.mp, L.np, L.kp, 1, cc, nullptr, 0, 0, rmax, cmax,
                     at<int8_t>(ws, L.part), L.part_bytes);
    }
  }
  {
    Scope sc(PH_SHIFTS, s);
    launch_shifts(s, rowbits, rmax, m, colbits, cmax, n, cc.Pprime, cc.c, at<int>(ws, L.mu_p),
                  at<int>(ws, L.nu_p), mu, nu, want_ef ? at<float>(ws, L.ef) : nullptr);
  }
  {
    Scope sc(PH_RES_A, s);
    launch_slices(s, pr, 1, true, A, lda, m, k, L.mp, L.kp, nullptr, mu, cc, As);
  }
  {
    Scope sc(PH_RES_B, s);
    launch_slices(s, pr, 1, false, B, ldb, n, k, L.np, L.kp, nullptr, nu, cc, Bs);
  }
  {
    Scope sc(PH_GEMM_RES, s);
    launch_gemm_i8(s, 0, As, (size_t)L.mp * L.kp, Bs, (size_t)L.np * L.kp, L.mp, L.np, L.kp,
                   cc.N, cc, W, (size_t)L.np * L.mp, L.mp, nullptr, nullptr, at<int8_t>(ws, L.part),
                   L.part_bytes);
  }
  {
    Scope sc(PH_CRT, s);
    launch_crt(s, pr, W, (size_t)L.np * L.mp, L.mp, mu, nu, m, n, cc, flag, C, ldc);
  }
  launch_or_status(s, flag, status);
  return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

int gemm_impl(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb, void* C,
              int ldc, int N, void* const* dbg) {
  const int b = pr == Prec::F64 ? 64 : 32;
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, true);
  if (rc) return rc;
  if ((rc = check_N(N, b))) return rc;
  if (m == 0 || n == 0) return OZAKI2_OK;
  hipStream_t s = g_stream;
  if (k == 0) {
    launch_fill_zero(s, pr, C, ldc, m, n);
    return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
  }
  CrtConsts cc;
  if ((rc = get_consts(N, b, &cc))) return rc;
  Layout L = layout(m, n, k, N, single_row_pad(m, n, N), N);
  char* ws;
  int* status;
  if ((rc = get_workspace(L.total, &ws, &status))) return rc;
  if (!dbg) return run_pipeline(pr, m, n, k, A, lda, B, ldb, C, ldc, cc, L, ws, status, s, false);
  rc = run_pipeline(pr, m, n, k, A, lda, B, ldb, C, ldc, cc, L, ws, status, s, true);
  if (rc || !dbg) return rc;
  // debug dumps (see ozaki2_debug_stages)
  auto cp = [&](void* dst, size_t off, size_t bytes) {
    if (dst && bytes) (void)hipMemcpyAsync(dst, ws + off, bytes, hipMemcpyDeviceToDevice, s);
  };
  cp(dbg[0], L.mu_p, 4ull * m);
  cp(dbg[1], L.nu_p, 4ull * n);
  cp(dbg[2], L.rmax, 4ull * m);
  cp(dbg[3], L.cmax, 4ull * n);
  cp(dbg[4], L.mu, 4ull * m);
  cp(dbg[5], L.nu, 4ull * n);
  for (int l = 0; l < N; ++l) {
    if (dbg[6])
      (void)hipMemcpy2DAsync((char*)dbg[6] + (size_t)l * m * k, k,
                             ws + L.A + (size_t)l * L.mp * L.kp, L.kp, k, m,
                             hipMemcpyDeviceToDevice, s);
    if (dbg[7])
      (void)hipMemcpy2DAsync((char*)dbg[7] + (size_t)l * n * k, k,
                             ws + L.B + (size_t)l * L.np * L.kp, L.kp, k, n,
                             hipMemcpyDeviceToDevice, s);
    if (dbg[8])
      (void)hipMemcpy2DAsync((char*)dbg[8] + (size_t)l * n * m, m,
                             ws + L.W + (size_t)l * L.np * L.mp, L.mp, m, n,
                             hipMemcpyDeviceToDevice, s);
  }
  if (dbg[10]) {
    cp(dbg[10], L.ef, 4ull * m);
    (void)hipMemcpyAsync((char*)dbg[10] + 4ull * m, ws + L.ef + 4ull * m, 4ull * n,
                         hipMemcpyDeviceToDevice, s);
  }
  // The INT32 residue products C'_l: the residue-product kernel with the
  // same tile choice, its accumulators stored instead of reduced mod p_l.
  if (dbg[11]) {
    int* D = nullptr;
    const size_t per = (size_t)L.np * L.mp;
    if (hipMalloc(&D, 4 * per * N) != hipSuccess) return OZAKI2_ERR_HIP;
    launch_gemm_i8(s, 4, at<int8_t>(ws, L.A), (size_t)L.mp * L.kp, at<int8_t>(ws, L.B),
                   (size_t)L.np * L.kp, L.mp, L.np, L.kp, N, cc, (int8_t*)D, per, L.mp, nullptr,
                   nullptr);
    for (int l = 0; l < N; ++l)
      (void)hipMemcpy2DAsync((char*)dbg[11] + 4ull * l * n * m, 4ull * m, D + l * per, 4ull * L.mp,
                             4ull * m, n, hipMemcpyDeviceToDevice, s);
    const bool ok = hipStreamSynchronize(s) == hipSuccess;
    (void)hipFree(D);
    if (!ok) return OZAKI2_ERR_HIP;
  }
  // C'(1), C'(2), Q and C'' from the CRT kernel's debug variant (it rewrites
  // the same C).
  if (dbg[12] || dbg[13] || dbg[14] || dbg[15]) {
    double* D = nullptr;
    const size_t mn = (size_t)m * n;
    if (hipMalloc(&D, 4 * 8 * mn) != hipSuccess) return OZAKI2_ERR_HIP;
    launch_crt_debug(s, pr, at<int8_t>(ws, L.W), (size_t)L.np * L.mp, L.mp, at<int>(ws, L.mu),
                     at<int>(ws, L.nu), m, n, cc, at<int>(ws, L.flag), C, ldc, D);
    for (int q = 0; q < 4; ++q)
      if (dbg[12 + q])
        (void)hipMemcpyAsync(dbg[12 + q], D + q * mn, 8 * mn, hipMemcpyDeviceToDevice, s);
    const bool ok = hipStreamSynchronize(s) == hipSuccess;
    (void)hipFree(D);
    if (!ok) return OZAKI2_ERR_HIP;
  }
  return hipStreamSynchronize(s) == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

// Complex C = AB (reading R23): the real Algorithm 1 on the embedding
// Ahat = [[Ar, -Ai], [Ai, Ar]] (2m x 2k), Bhat = [[Br], [Bi]] (2k x n),
// whose product holds Re AB in rows 1..m and Im AB in rows m+1..2m; the CRT
// writes the two halves as complex pairs.  The workspace holds Ahat and
// Bhat, then the real layout of the 2m x n x 2k problem.
// The real embedding of a complex product, formed in place by the slice
// kernels: Ahat = [[Ar, -Ai], [Ai, Ar]] with its k halves kh = rup(k, 128)
// apart and its row halves half = mp / 2 apart (zero rows and columns
// between them change no product, maximum or shift), Bhat = [[Br], [Bi]]
// with the same k halves.  The layout is the real one of the
// 2 half x n x 2 kh problem.
struct ZLayout {
  int kh, half;
  Layout L;
};

ZLayout zlayout(int m, int n, int k, int N) {
  ZLayout Z;
  Z.kh = (int)rup((size_t)k, 128);
  Z.L = layout(2 * m, n, 2 * Z.kh, N, single_row_pad(2 * m, n, N), N);
  Z.half = Z.L.mp / 2;
  return Z;
}

// Argument checks of the complex calls (leading dimensions in complex
// elements).  kmax: the largest k of the form (the embedding doubles k; the
// 3-product form keeps it).  needC: the call writes C (the planner does not).
int check_complex_args(int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                       const void* C, int ldc, int kmax, bool needC = true) {
  if (m < 0 || n < 0 || k < 0 || m > kMaxDim / 2 || n > kMaxDim) return OZAKI2_ERR_INVALID_ARG;
  if (lda < (m > 1 ? m : 1) || ldb < (k > 1 ? k : 1)) return OZAKI2_ERR_INVALID_ARG;
  if (needC && (ldc < (m > 1 ? m : 1) || ldc > INT32_MAX / 2)) return OZAKI2_ERR_INVALID_ARG;
  if ((size_t)m * k > 0 && !A) return OZAKI2_ERR_INVALID_ARG;
  if ((size_t)k * n > 0 && !B) return OZAKI2_ERR_INVALID_ARG;
  if (needC && (size_t)m * n > 0 && !C) return OZAKI2_ERR_INVALID_ARG;
  if (k > kmax) return OZAKI2_ERR_K_RANGE;
  return OZAKI2_OK;
}

int zgemm_impl(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
               void* C, int ldc, int N) {
  const int b = pr == Prec::F64 ? 64 : 32;
  int rc = check_complex_args(m, n, k, A, lda, B, ldb, C, ldc, kMaxK / 2);
  if (rc) return rc;
  if ((rc = check_N(N, b))) return rc;
  if (m == 0 || n == 0) return OZAKI2_OK;
  hipStream_t s = g_stream;
  if (k == 0) {  // C = 0: the interleaved pairs as a 2m x n real matrix
    launch_fill_zero(s, pr, C, 2 * ldc, 2 * m, n);
    return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
  }
  CrtConsts cc;
  if ((rc = get_consts(N, b, &cc))) return rc;
  const ZLayout Z = zlayout(m, n, k, N);
  const Layout& L = Z.L;
  char* ws;
  int* status;
  if ((rc = get_workspace(L.total, &ws, &status))) return rc;
  uint64_t* rowbits = at<uint64_t>(ws, L.rowbits);
  uint64_t* colbits = at<uint64_t>(ws, L.colbits);
  int* rmax = at<int>(ws, L.rmax);
  int* cmax = at<int>(ws, L.cmax);
  int* flag = at<int>(ws, L.flag);
  int* mu = at<int>(ws, L.mu);
  int* nu = at<int>(ws, L.nu);
  int8_t* As = at<int8_t>(ws, L.A);
  int8_t* Bs = at<int8_t>(ws, L.B);
  int8_t* W = at<int8_t>(ws, L.W);
  const int H = Z.half;
  // Algorithm 2 on the embedding: the row maxima of Ahat's rows i and H + i
  // are both the complex row's maximum over its two parts; a column of Bhat
  // holds both parts of a column of B.
  launch_init(s, rowbits, L.mp, colbits, L.np, rmax, cmax, flag);
  launch_absmax_rows(s, pr, A, lda, m, k, rowbits, flag, true, H);
  launch_absmax_cols(s, pr, B, ldb, k, n, colbits, flag, true);
  launch_slices_embed(s, pr, 0, true, A, lda, m, k, Z.kh, L.mp, H, rowbits, nullptr, cc, As);
  launch_slices_embed(s, pr, 0, false, B, ldb, n, k, Z.kh, L.np, 0, colbits, nullptr, cc, Bs);
  launch_gemm_i8(s, 1, As, 0, Bs, 0, L.mp, L.np, L.kp, 1, cc, nullptr, 0, 0, rmax, cmax,
                 at<int8_t>(ws, L.part), L.part_bytes);
  launch_shifts(s, rowbits, rmax, L.mp, colbits, cmax, n, cc.Pprime, cc.c, at<int>(ws, L.mu_p),
                at<int>(ws, L.nu_p), mu, nu, nullptr);
  // Algorithm 3 on the embedding, its residues formed from the complex
  // source; the CRT writes rows i (real) and H + i (imaginary) as pairs.
  launch_slices_embed(s, pr, 1, true, A, lda, m, k, Z.kh, L.mp, H, nullptr, mu, cc, As);
  launch_slices_embed(s, pr, 1, false, B, ldb, n, k, Z.kh, L.np, 0, nullptr, nu, cc, Bs);
  launch_gemm_i8(s, 0, As, (size_t)L.mp * L.kp, Bs, (size_t)L.np * L.kp, L.mp, L.np, L.kp, N, cc,
                 W, (size_t)L.np * L.mp, L.mp, nullptr, nullptr, at<int8_t>(ws, L.part),
                 L.part_bytes);
  launch_crt_complex(s, pr, W, W + H, (size_t)L.np * L.mp, L.mp, mu, mu + H, nu, m, n, cc, flag, C,
                     ldc);
  launch_or_status(s, flag, status);
  return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

// The complex 3-product form (reading R25): one shift per row of A and per
// column of B for both parts (Algorithm 2 on Abar = bar(Ar) + bar(Ai) with
// mu' one lower), residues of A'r, A'i and A'r + A'i, three residue products
// per modulus, W_re = mod(T1 - T2), W_im = mod(T3 - T1 - T2), the CRT on
// each part and the inverse scaling, written as complex pairs.  The kernels
// read the interleaved complex inputs in place, so the workspace is the
// layout of the m x n x k problem with 3N slices and 3N W (the three groups
// of N back to back).
struct Z3Layout {
  size_t total;
  Layout L;
};

Z3Layout z3layout(int m, int n, int k, int N) {
  Z3Layout Z;
  Z.L = layout(m, n, k, 3 * N, single_row_pad(m, n, N), N);
  Z.total = Z.L.total;
  return Z;
}

int zgemm3m_impl(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                 void* C, int ldc, int N) {
  const int b = pr == Prec::F64 ? 64 : 32;
  int rc = check_complex_args(m, n, k, A, lda, B, ldb, C, ldc, kMaxK);
  if (rc) return rc;
  if ((rc = check_N(N, b))) return rc;
  if (m == 0 || n == 0) return OZAKI2_OK;
  hipStream_t s = g_stream;
  if (k == 0) {
    launch_fill_zero(s, pr, C, 2 * ldc, 2 * m, n);
    return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
  }
  CrtConsts cc;
  if ((rc = get_consts(N, b, &cc))) return rc;
  const Z3Layout Z = z3layout(m, n, k, N);
  char* ws;
  int* status;
  if ((rc = get_workspace(Z.total, &ws, &status))) return rc;
  const Layout& L = Z.L;
  char* w = ws;
  uint64_t* rowbits = at<uint64_t>(w, L.rowbits);
  uint64_t* colbits = at<uint64_t>(w, L.colbits);
  int* rmax = at<int>(w, L.rmax);
  int* cmax = at<int>(w, L.cmax);
  int* flag = at<int>(w, L.flag);
  int* mu = at<int>(w, L.mu);
  int* nu = at<int>(w, L.nu);
  const size_t sa = (size_t)L.mp * L.kp, sb = (size_t)L.np * L.kp, sw = (size_t)L.np * L.mp;
  int8_t* X[3] = {at<int8_t>(w, L.A), at<int8_t>(w, L.A) + N * sa, at<int8_t>(w, L.A) + 2 * N * sa};
  int8_t* Y[3] = {at<int8_t>(w, L.B), at<int8_t>(w, L.B) + N * sb, at<int8_t>(w, L.B) + 2 * N * sb};
  int8_t* W[3] = {at<int8_t>(w, L.W), at<int8_t>(w, L.W) + N * sw, at<int8_t>(w, L.W) + 2 * N * sw};
  // Algorithm 2 on the complex matrices, read in place: abs-max over both
  // parts, and Abar = bar(Ar) + bar(Ai) (Bbar alike) into the third set.
  launch_init(s, rowbits, L.mp, colbits, L.np, rmax, cmax, flag);
  launch_absmax_rows(s, pr, A, lda, m, k, rowbits, flag, true);
  launch_absmax_cols(s, pr, B, ldb, k, n, colbits, flag, true);
  launch_slices_complex(s, pr, 2, true, A, lda, m, k, L.mp, L.kp, rowbits, nullptr, cc, X[2]);
  launch_slices_complex(s, pr, 2, false, B, ldb, n, k, L.np, L.kp, colbits, nullptr, cc, Y[2]);
  launch_gemm_i8(s, 1, X[2], 0, Y[2], 0, L.mp, L.np, L.kp, 1, cc, nullptr, 0, 0, rmax, cmax,
                 at<int8_t>(w, L.part), L.part_bytes);
  launch_shifts(s, rowbits, rmax, m, colbits, cmax, n, cc.Pprime, cc.c, at<int>(w, L.mu_p),
                at<int>(w, L.nu_p), mu, nu, nullptr, -1);
  // Algorithm 3: residues of A'r, A'i and A'r + A'i (and of B) in one pass
  // per operand, three residue products per modulus, and the CRT of the real
  // and imaginary residues formed from the three W.
  launch_slices_complex(s, pr, 1, true, A, lda, m, k, L.mp, L.kp, nullptr, mu, cc, X[0]);
  launch_slices_complex(s, pr, 1, false, B, ldb, n, k, L.np, L.kp, nullptr, nu, cc, Y[0]);
  for (int q = 0; q < 3; ++q)
    launch_gemm_i8(s, 0, X[q], sa, Y[q], sb, L.mp, L.np, L.kp, N, cc, W[q], sw, L.mp, nullptr,
                   nullptr, at<int8_t>(w, L.part), L.part_bytes);
  launch_crt_3m(s, pr, W[0], W[1], W[2], sw, L.mp, mu, nu, m, n, cc, flag, C, ldc);
  launch_or_status(s, flag, status);
  return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

}  // namespace

namespace oz2 {

// Algorithm 1 for one problem with the workspace `ws` (capacity `cap`
// bytes) and status word `status` that the caller provides; allocates
// nothing.  The size check comes before any HIP call.
int gemm_on_buffer(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                   void* C, int ldc, int N, size_t cap, BufferSource get) {
  const int b = pr == Prec::F64 ? 64 : 32;
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, true);
  if (rc) return rc;
  if ((rc = check_N(N, b))) return rc;
  if (m == 0 || n == 0) return OZAKI2_OK;
  const Layout L = layout(m, n, k > 0 ? k : 1, N, single_row_pad(m, n, N), N);
  if (L.total > cap) return OZAKI2_ERR_WORKSPACE;
  hipStream_t s = g_stream;
  if (k == 0) {
    launch_fill_zero(s, pr, C, ldc, m, n);
    return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
  }
  CrtConsts cc;
  if ((rc = get_consts(N, b, &cc))) return rc;
  char* ws = nullptr;
  int* status = nullptr;
  if ((rc = get(&ws, &status))) return rc;
  return run_pipeline(pr, m, n, k, A, lda, B, ldb, C, ldc, cc, L, ws, status, s, false);
}

}  // namespace oz2

namespace {

// ---------------------------------------------------------------------------
// batched execution: every phase of Algorithm 1 is one grouped launch over all
// problems of the batch (a device table of problem descriptors plus, per
// phase, a prefix array of workgroup counts).  The launch sequence is captured
// once per batch signature into a hipGraph and replayed on later calls.
// ---------------------------------------------------------------------------
// BS_ABB: abs-max of B with Bbar in one read (k_pad <= kAbsBarMaxK);
// BS_ABS_B and BS_BAR_B: the two passes for the other problems; BS_SL_B: the
// residues of B for every problem.
enum BatchSlot {
  BS_INIT, BS_ABS_A, BS_ABS_B, BS_ABB, BS_SL_A, BS_BAR_B, BS_SL_B, BS_GS_BIG, BS_GS_SMALL,
  BS_SHIFTS, BS_GR_BIG, BS_GR_SMALL, BS_CRT, BS_COUNT
};
constexpr int kMaxBatchEntries = 8;

struct BatchEntry {
  int dev = 0;                           // device holding the resources below
  std::vector<int64_t> key;
  char* table = nullptr;                 // device: descriptors, then one block map per slot
  size_t table_bytes = 0;                // allocated size
  std::vector<int> zero_fill;            // problems with k = 0 (C := 0)
  int active = 0;                        // problems with m, n, k >= 1
  int blocks[BS_COUNT] = {};             // grid size per slot
  size_t map_off[BS_COUNT] = {};         // byte offset of each slot's block map
  int split = 0;                         // problems with >= split 256x256 tiles use them
  bool persist = false;                  // residue products: persistent kernels
  // One launch per problem for the scaling and residue products (the
  // single-problem launcher, which splits k where a problem's output leaves
  // the GPU idle), for batches of at most kPerProblemMax problems.
  bool per_problem = false;
  std::vector<ProbDesc> hd;              // host copies of the descriptors
  std::vector<CrtConsts> hc;             // constants of each problem's N
  std::vector<int8_t*> part;             // split-k scratch of each problem (may be empty)
  std::vector<size_t> part_bytes;
  bool fold = false;                     // some k_pad > 2^17 (reduction mod p inside k)
  int pgrid[2] = {0, 0};                 // resident workgroups of the persistent kernels (256, 128)
  int res_path = -1;                     // residue path code for the grouped slice kernels
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // The last reference may drop while a replay is still running: wait for
  // the entry's device before releasing the graph and the table.
  ~BatchEntry() {
    if (!exec && !graph && !table) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (table) (void)hipFree(table);
    if (cur != dev) (void)hipSetDevice(cur);
  }
};

// Batch knobs (ozaki2_debug_tuning): a forced tile split (-1: autotune),
// whether a batch's launch sequence is captured into a hipGraph, and a forced
// form of the residue products (-1: autotune, 0: one workgroup per tile,
// 1: persistent).
std::atomic<int> g_batch_split{-1};
std::atomic<int> g_batch_graph{1};
std::atomic<int> g_batch_persist{-1};
constexpr int kPerProblemMax = 64;   // batches up to this many problems may run per problem

// Device table of CrtConsts indexed by N (entries below 2 unused).
int get_ctab(int b, CrtConsts** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  const int nmax = b == 64 ? kMaxModuli : 16;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    CrtConsts* t = g_dev[dev].ctab[g_table][b == 64 ? 0 : 1];
    if (t) {
      *out = t;
      return OZAKI2_OK;
    }
  }
  std::vector<CrtConsts> host(kMaxModuli + 1);
  memset(host.data(), 0, host.size() * sizeof(CrtConsts));
  for (int N = 2; N <= nmax; ++N) {
    int rc = get_consts(N, b, &host[N]);
    if (rc) return rc;
  }
  CrtConsts* t = nullptr;
  if (hipMalloc(&t, host.size() * sizeof(CrtConsts)) != hipSuccess) return OZAKI2_ERR_HIP;
  if (hipMemcpy(t, host.data(), host.size() * sizeof(CrtConsts), hipMemcpyHostToDevice) !=
      hipSuccess)
    return OZAKI2_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  CrtConsts*& slot = g_dev[dev].ctab[g_table][b == 64 ? 0 : 1];
  if (slot) {
    (void)hipFree(t);   // another thread got there first
  } else {
    slot = t;
  }
  *out = slot;
  return OZAKI2_OK;
}

// Problem descriptors and per-slot block maps for the active problems, with
// the tile split `split` (problems with at least `split` 256x256 tiles per
// product use the 256x256 kernel, the rest 128x128; 0 = all 256x256).
void build_table(const std::vector<ProbDesc>& D, int split, std::vector<char>* out,
                 int blocks[BS_COUNT], size_t map_off[BS_COUNT]) {
  const int cnt = (int)D.size();
  std::vector<int> c((size_t)BS_COUNT * cnt);
  for (int p = 0; p < cnt; ++p) {
    const ProbDesc& d = D[p];
    const bool big = d.mp % 256 == 0 && d.np % 256 == 0 &&
                     (int64_t)(d.mp / 256) * (d.np / 256) >= split;
    int* cp = &c[(size_t)p * BS_COUNT];
    cp[BS_INIT] = group_init_blocks(d.mp, d.np);
    cp[BS_ABS_A] = cdiv_i(d.m, 256) * cdiv_i(d.k, 64);
    const bool fuse_b = d.kp <= kAbsBarMaxK;
    cp[BS_ABS_B] = fuse_b ? 0 : absmax_cols_blocks(d.n);
    cp[BS_ABB] = fuse_b ? absbar_group_blocks(d.np, d.kp) : 0;
    cp[BS_SL_A] = (d.kp / 128) * (d.mp / 32);
    cp[BS_BAR_B] = fuse_b ? 0 : (d.kp / 128) * (d.np / 32);
    cp[BS_SL_B] = (d.kp / 128) * (d.np / 32);
    cp[BS_GS_BIG] = big ? group_gemm_blocks(d.mp, d.np, 256, 1) : 0;
    cp[BS_GS_SMALL] = big ? 0 : group_gemm_blocks(d.mp, d.np, 128, 1);
    cp[BS_SHIFTS] = cdiv_i(d.m + d.n, 256);
    cp[BS_GR_BIG] = big ? group_gemm_blocks(d.mp, d.np, 256, d.N) : 0;
    cp[BS_GR_SMALL] = big ? 0 : group_gemm_blocks(d.mp, d.np, 128, d.N);
    cp[BS_CRT] = (int)crt_blocks(d.m, d.n);
  }
  size_t off = rup(sizeof(ProbDesc) * cnt, 256);
  for (int sl = 0; sl < BS_COUNT; ++sl) {
    int64_t tot = 0;
    for (int p = 0; p < cnt; ++p) tot += c[(size_t)p * BS_COUNT + sl];
    blocks[sl] = tot > 0x7FFFFFFF ? -1 : (int)tot;
    map_off[sl] = off;
    off += rup(sizeof(BlockRef) * (size_t)tot, 256);
  }
  out->assign(off, 0);
  memcpy(out->data(), D.data(), sizeof(ProbDesc) * cnt);
  // The residue-product maps list the problems by decreasing k, so that the
  // persistent kernels, which deal entries out in a fixed stride, start with
  // the longest tiles and end with the shortest (each problem's entries stay
  // a multiple of 8 long, so every entry keeps its XCD).
  std::vector<int> by_k(cnt);
  for (int p = 0; p < cnt; ++p) by_k[p] = p;
  std::stable_sort(by_k.begin(), by_k.end(), [&](int a, int b) { return D[a].kp > D[b].kp; });
  for (int sl = 0; sl < BS_COUNT; ++sl) {
    BlockRef* map = reinterpret_cast<BlockRef*>(out->data() + map_off[sl]);
    const bool sorted = sl == BS_GR_BIG || sl == BS_GR_SMALL;
    size_t q = 0;
    for (int t = 0; t < cnt; ++t) {
      const int p = sorted ? by_k[t] : t;
      for (int l = 0; l < c[(size_t)p * BS_COUNT + sl]; ++l) map[q++] = BlockRef{p, l};
    }
  }
}

// Grid sizes over 2^31 - 1 cannot be launched.
bool table_fits(const int blocks[BS_COUNT]) {
  for (int sl = 0; sl < BS_COUNT; ++sl)
    if (blocks[sl] < 0) return false;
  return true;
}

// The residue products of a batch, in the entry's form.
void enqueue_residue_products(const BatchEntry& e, const CrtConsts* ctab, hipStream_t s) {
  if (e.per_problem) {
    for (size_t q = 0; q < e.hd.size(); ++q) {
      const ProbDesc& d = e.hd[q];
      launch_gemm_i8(s, 0, d.As, (size_t)d.mp * d.kp, d.Bs, (size_t)d.np * d.kp, d.mp, d.np, d.kp,
                     d.N, e.hc[q], d.W, (size_t)d.np * d.mp, d.mp, nullptr, nullptr, e.part[q],
                     e.part_bytes[q]);
    }
    return;
  }
  const ProbDesc* D = reinterpret_cast<const ProbDesc*>(e.table);
  auto M = [&](int sl) { return reinterpret_cast<const BlockRef*>(e.table + e.map_off[sl]); };
  if (e.persist) {
    launch_group_gemm_persist(s, 256, e.fold, e.pgrid[0], D, M(BS_GR_BIG), e.blocks[BS_GR_BIG],
                              ctab);
    launch_group_gemm_persist(s, 128, e.fold, e.pgrid[1], D, M(BS_GR_SMALL),
                              e.blocks[BS_GR_SMALL], ctab);
  } else {
    launch_group_gemm(s, 0, 256, D, M(BS_GR_BIG), e.blocks[BS_GR_BIG], ctab);
    launch_group_gemm(s, 0, 128, D, M(BS_GR_SMALL), e.blocks[BS_GR_SMALL], ctab);
  }
}

// Enqueue the grouped launch sequence on `s` (table already on the device).
void enqueue_batch(Prec pr, const BatchEntry& e, const CrtConsts* ctab, int* status, hipStream_t s,
                   void* const* C, const int* ldc, const int* mnkN) {
  const ProbDesc* D = reinterpret_cast<const ProbDesc*>(e.table);
  auto M = [&](int sl) { return reinterpret_cast<const BlockRef*>(e.table + e.map_off[sl]); };
  auto B = [&](int sl) { return e.blocks[sl]; };
  for (int p : e.zero_fill) launch_fill_zero(s, pr, C[p], ldc[p], mnkN[4 * p], mnkN[4 * p + 1]);
  if (e.active == 0) return;
  launch_group_scale(s, pr, GP_INIT, D, M(BS_INIT), B(BS_INIT), ctab);
  launch_group_scale(s, pr, GP_ABSMAX_A, D, M(BS_ABS_A), B(BS_ABS_A), ctab);
  launch_group_scale(s, pr, GP_ABSMAX_B, D, M(BS_ABS_B), B(BS_ABS_B), ctab);
  launch_group_scale(s, pr, GP_ABSBAR_B, D, M(BS_ABB), B(BS_ABB), ctab);
  launch_group_slices(s, pr, 0, true, -1, D, M(BS_SL_A), B(BS_SL_A), ctab);
  launch_group_slices(s, pr, 0, false, -1, D, M(BS_BAR_B), B(BS_BAR_B), ctab);
  if (e.per_problem) {
    for (size_t q = 0; q < e.hd.size(); ++q) {
      const ProbDesc& d = e.hd[q];
      launch_gemm_i8(s, 1, d.As, 0, d.Bs, 0, d.mp, d.np, d.kp, 1, e.hc[q], nullptr, 0, 0, d.rmax,
                     d.cmax, e.part[q], e.part_bytes[q]);
    }
  } else {
    launch_group_gemm(s, 1, 256, D, M(BS_GS_BIG), B(BS_GS_BIG), ctab);
    launch_group_gemm(s, 1, 128, D, M(BS_GS_SMALL), B(BS_GS_SMALL), ctab);
  }
  launch_group_scale(s, pr, GP_SHIFTS, D, M(BS_SHIFTS), B(BS_SHIFTS), ctab);
  launch_group_slices(s, pr, 1, true, e.res_path, D, M(BS_SL_A), B(BS_SL_A), ctab);
  launch_group_slices(s, pr, 1, false, e.res_path, D, M(BS_SL_B), B(BS_SL_B), ctab);
  enqueue_residue_products(e, ctab, s);
  launch_group_crt(s, pr, D, M(BS_CRT), B(BS_CRT), e.active, ctab, status);
}

// Copies a host table to the entry's device table, growing it if needed.
int upload_table(BatchEntry* e, const std::vector<char>& host, hipStream_t s) {
  if (hipStreamSynchronize(s) != hipSuccess) return OZAKI2_ERR_HIP;
  if (host.empty()) return OZAKI2_OK;
  if (host.size() > e->table_bytes) {
    if (e->table) (void)hipFree(e->table);
    e->table = nullptr;
    e->table_bytes = 0;
    if (hipMalloc(&e->table, host.size()) != hipSuccess) return OZAKI2_ERR_HIP;
    e->table_bytes = host.size();
  }
  if (hipMemcpy(e->table, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return OZAKI2_ERR_HIP;
  return OZAKI2_OK;
}

// Autotuner: times the residue products (the dominant phase) under each
// candidate tile split and form (one workgroup per tile, persistent, or,
// where some problem has split-k scratch, one launch per problem) and keeps
// the fastest; the form chosen also applies to the scaling products.  The caller has run the whole batch once, so the
// operand slices in the workspace are this batch's own residues; the split
// does not move them (the padding of every problem is fixed).  A forced
// split or form (forced_split >= 0, forced_persist >= 0) is not tuned.
int tune_batch(const std::vector<ProbDesc>& D, BatchEntry* e, const CrtConsts* ctab,
               hipStream_t s, int forced_split, int forced_persist) {
  std::vector<int> splits = forced_split >= 0 ? std::vector<int>{forced_split}
                                              : std::vector<int>{1 << 30, 16, 4, 0};
  // form 2 (one launch per problem) only where some problem splits its k
  bool any_part = false;
  for (size_t q = 0; q < e->part_bytes.size(); ++q) any_part = any_part || e->part_bytes[q] > 0;
  std::vector<int> forms = forced_persist >= 0 ? std::vector<int>{forced_persist}
                                               : (any_part ? std::vector<int>{1, 0, 2}
                                                           : std::vector<int>{1, 0});
  float best_ms = 0.f;
  bool have = false;
  int best_split = splits[0], best_form = forms[0];
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return OZAKI2_ERR_HIP;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return OZAKI2_ERR_HIP;
  }
  int rc = OZAKI2_OK;
  std::vector<char> host;
  for (size_t c = 0; c < splits.size() && rc == OZAKI2_OK; ++c) {
    build_table(D, splits[c], &host, e->blocks, e->map_off);
    if (!table_fits(e->blocks)) continue;
    if ((rc = upload_table(e, host, s))) break;
    for (int form : forms) {
      if (form == 2 && c > 0) continue;   // tile splits do not apply to the per-problem form
      e->persist = form == 1;
      e->per_problem = form == 2;
      float ms = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        if (rep == 1) (void)hipEventRecord(a, s);
        enqueue_residue_products(*e, ctab, s);
      }
      (void)hipEventRecord(b, s);
      if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        rc = OZAKI2_ERR_HIP;
        break;
      }
      if (!have || ms < best_ms) {
        have = true;
        best_ms = ms;
        best_split = splits[c];
        best_form = form;
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  e->split = best_split;
  e->persist = best_form == 1;
  e->per_problem = best_form == 2;
  return rc;
}

// Workspace of a batch: the layouts of the active problems (m, n, k >= 1),
// back to back; their indices and offsets go to act / off.
// A batch of at most kPerProblemMax active problems also holds each
// problem's split-k scratch (none for problems whose output fills the GPU),
// for the per-problem form of the products.
bool batch_per_problem_ok(int count, const int* mnkN) {
  int active = 0;
  for (int p = 0; p < count; ++p)
    active += mnkN[4 * p] > 0 && mnkN[4 * p + 1] > 0 && mnkN[4 * p + 2] > 0;
  return active <= kPerProblemMax;
}

Layout batch_problem_layout(int m, int n, int k, int N, bool per_problem) {
  return layout(m, n, k, N, batch_row_pad(m, n), per_problem ? N : 0);
}

size_t batch_layout(int count, const int* mnkN, std::vector<int>* act, std::vector<size_t>* off) {
  const bool pp = batch_per_problem_ok(count, mnkN);
  size_t total = 0;
  for (int p = 0; p < count; ++p) {
    const int m = mnkN[4 * p], n = mnkN[4 * p + 1], k = mnkN[4 * p + 2];
    if (m == 0 || n == 0 || k == 0) continue;
    if (act) act->push_back(p);
    if (off) off->push_back(total);
    total += rup(batch_problem_layout(m, n, k, mnkN[4 * p + 3], pp).total, 256);
  }
  return total;
}

int batched_impl(Prec pr, int count, const int* mnkN, const void* const* A, const int* lda,
                 const void* const* B, const int* ldb, void* const* C, const int* ldc) {
  const int b = pr == Prec::F64 ? 64 : 32;
  for (int p = 0; p < count; ++p) {
    int rc = check_args(mnkN[4 * p], mnkN[4 * p + 1], mnkN[4 * p + 2], A[p], lda[p], B[p], ldb[p],
                        C[p], ldc[p], true);
    if (rc) return rc;
    if ((rc = check_N(mnkN[4 * p + 3], b))) return rc;
  }
  hipStream_t s = g_stream;
  std::vector<int> act;
  std::vector<size_t> off;
  const size_t total = batch_layout(count, mnkN, &act, &off);
  const bool pp = batch_per_problem_ok(count, mnkN);
  char* ws = nullptr;
  int* status = nullptr;
  uint64_t gen = 0;
  int rc = get_workspace(total, &ws, &status, &gen);
  if (rc) return rc;
  CrtConsts* ctab = nullptr;
  if ((rc = get_ctab(b, &ctab))) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;

  const int forced = g_batch_split.load(std::memory_order_relaxed);
  const int forced_persist = g_batch_persist.load(std::memory_order_relaxed);
  const bool use_graph = g_batch_graph.load(std::memory_order_relaxed) != 0;
  std::vector<int64_t> key;
  key.reserve(4 + 10 * (size_t)count);
  key.push_back(b);
  key.push_back(g_table);
  key.push_back((int64_t)(intptr_t)ws);
  key.push_back((int64_t)gen);
  key.push_back(forced);
  key.push_back(forced_persist);
  key.push_back(use_graph ? 1 : 0);
  key.push_back(g_split_k.load(std::memory_order_relaxed));   // captured split-k choices
  for (int p = 0; p < count; ++p) {
    for (int q = 0; q < 4; ++q) key.push_back(mnkN[4 * p + q]);
    key.push_back(lda[p]);
    key.push_back(ldb[p]);
    key.push_back(ldc[p]);
    key.push_back((int64_t)(intptr_t)A[p]);
    key.push_back((int64_t)(intptr_t)B[p]);
    key.push_back((int64_t)(intptr_t)C[p]);
  }

  std::shared_ptr<BatchEntry> e;   // keeps the entry alive while it is used
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& x : g_dev[dev].batches)
      if (x->key == key) e = x;
  }
  if (!e) {
    e = std::make_shared<BatchEntry>();
    e->dev = dev;
    e->key = key;
    e->active = (int)act.size();
    for (int p = 0; p < count; ++p)
      if (mnkN[4 * p] > 0 && mnkN[4 * p + 1] > 0 && mnkN[4 * p + 2] == 0) e->zero_fill.push_back(p);
    std::vector<ProbDesc> D(act.size());
    for (size_t q = 0; q < act.size(); ++q) {
      const int p = act[q];
      const int m = mnkN[4 * p], n = mnkN[4 * p + 1], k = mnkN[4 * p + 2], N = mnkN[4 * p + 3];
      const Layout L = batch_problem_layout(m, n, k, N, pp);
      char* w = ws + off[q];
      e->part.push_back(L.part_bytes ? at<int8_t>(w, L.part) : nullptr);
      e->part_bytes.push_back(L.part_bytes);
      ProbDesc& d = D[q];
      d.m = m, d.n = n, d.k = k, d.N = N;
      d.mp = L.mp, d.np = L.np, d.kp = L.kp;
      d.lda = lda[p], d.ldb = ldb[p], d.ldc = ldc[p];
      d.A = A[p], d.B = B[p], d.C = C[p];
      d.rowbits = at<uint64_t>(w, L.rowbits);
      d.colbits = at<uint64_t>(w, L.colbits);
      d.rmax = at<int>(w, L.rmax);
      d.cmax = at<int>(w, L.cmax);
      d.mu = at<int>(w, L.mu);
      d.nu = at<int>(w, L.nu);
      d.flag = at<int>(w, L.flag);
      d.As = at<int8_t>(w, L.A);
      d.Bs = at<int8_t>(w, L.B);
      d.W = at<int8_t>(w, L.W);
      e->hc.emplace_back();
      if ((rc = get_consts(N, b, &e->hc.back()))) return rc;
    }
    e->hd = D;
    {
      // one residue kernel for the whole batch when every N takes the same path
      std::vector<CrtConsts> cs;
      std::vector<int> seen;
      for (const ProbDesc& d : D) {
        if (std::find(seen.begin(), seen.end(), d.N) != seen.end()) continue;
        seen.push_back(d.N);
        cs.emplace_back();
        if ((rc = get_consts(d.N, pr == Prec::F64 ? 64 : 32, &cs.back()))) return rc;
      }
      std::vector<const CrtConsts*> ptrs;
      for (const CrtConsts& c : cs) ptrs.push_back(&c);
      e->res_path = group_residue_path(ptrs.data(), (int)ptrs.size());
    }
    for (const ProbDesc& d : D) e->fold = e->fold || d.kp > (1 << 17);
    e->pgrid[0] = persist_grid(256);
    e->pgrid[1] = persist_grid(128);
    std::vector<char> host;
    e->split = forced >= 0 ? forced : 1 << 30;
    e->persist = forced_persist == 1 || forced_persist < 0;
    e->per_problem = forced_persist == 2;
    if ((forced < 0 || forced_persist < 0) && e->active > 0) {
      // One eager pass of the whole batch first, so that the tuner times the
      // residue products on this batch's own residues.
      build_table(D, e->split, &host, e->blocks, e->map_off);
      if (!table_fits(e->blocks)) return OZAKI2_ERR_INVALID_ARG;
      if ((rc = upload_table(e.get(), host, s))) return rc;
      enqueue_batch(pr, *e, ctab, status, s, C, ldc, mnkN);
      if ((rc = tune_batch(D, e.get(), ctab, s, forced, forced_persist))) return rc;
    }
    build_table(D, e->split, &host, e->blocks, e->map_off);
    if (!table_fits(e->blocks)) return OZAKI2_ERR_INVALID_ARG;
    if ((rc = upload_table(e.get(), host, s))) return rc;
    if (use_graph) {
      hipStream_t cs;
      {
        std::lock_guard<std::mutex> lk(g_mu);
        cs = g_dev[dev].capture;
      }
      if (!cs) {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
          return OZAKI2_ERR_HIP;
        std::lock_guard<std::mutex> lk(g_mu);
        g_dev[dev].capture = cs;
      }
      bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        enqueue_batch(pr, *e, ctab, status, cs, C, ldc, mnkN);
        ok = hipStreamEndCapture(cs, &e->graph) == hipSuccess && e->graph;
      }
      if (ok) ok = hipGraphInstantiateWithFlags(&e->exec, e->graph, 0) == hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        return OZAKI2_ERR_HIP;
      }
    }
    std::vector<std::shared_ptr<BatchEntry>> evict;   // released outside the lock
    {
      std::lock_guard<std::mutex> lk(g_mu);
      auto& v = g_dev[dev].batches;
      v.push_back(e);
      while ((int)v.size() > kMaxBatchEntries) {
        evict.push_back(v.front());
        v.erase(v.begin());
      }
    }
  }
  Scope sc(PH_BATCH, s);
  if (e->exec) {
    if (hipGraphLaunch(e->exec, s) != hipSuccess) return OZAKI2_ERR_HIP;
  } else {
    enqueue_batch(pr, *e, ctab, status, s, C, ldc, mnkN);
  }
  return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

}  // namespace

extern "C" {

int ozaki2_gemm(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C,
                int ldc, int N) {
  return gemm_impl(Prec::F64, m, n, k, A, lda, B, ldb, C, ldc, N, nullptr);
}

int ozaki2_sgemm(int m, int n, int k, const float* A, int lda, const float* B, int ldb, float* C,
                 int ldc, int N) {
  return gemm_impl(Prec::F32, m, n, k, A, lda, B, ldb, C, ldc, N, nullptr);
}

int ozaki2_zgemm(int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                 double* C, int ldc, int N) {
  return zgemm_impl(Prec::F64, m, n, k, A, lda, B, ldb, C, ldc, N);
}

int ozaki2_cgemm(int m, int n, int k, const float* A, int lda, const float* B, int ldb, float* C,
                 int ldc, int N) {
  return zgemm_impl(Prec::F32, m, n, k, A, lda, B, ldb, C, ldc, N);
}

int ozaki2_zgemm3m(int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                   double* C, int ldc, int N) {
  return zgemm3m_impl(Prec::F64, m, n, k, A, lda, B, ldb, C, ldc, N);
}

int ozaki2_cgemm3m(int m, int n, int k, const float* A, int lda, const float* B, int ldb,
                   float* C, int ldc, int N) {
  return zgemm3m_impl(Prec::F32, m, n, k, A, lda, B, ldb, C, ldc, N);
}

size_t ozaki2_complex_workspace_bytes(int prec, int m, int n, int k, int N) {
  if ((prec != 64 && prec != 32) || m < 0 || n < 0 || k < 0) return 0;
  if (m > kMaxDim / 2 || n > kMaxDim || k > kMaxK || check_N(N, prec) != OZAKI2_OK) return 0;
  if (m == 0 || n == 0 || k == 0) return 0;
  const size_t s = prec == 64 ? 8 : 4;
  const size_t t3 = z3layout(m, n, k, N).total;
  if (k > kMaxK / 2) return t3;   // only the 3-product form takes such k
  const size_t t4 = zlayout(m, n, k, N).L.total;
  return t3 > t4 ? t3 : t4;
}

int ozaki2_set_stream(void* stream) {
  g_stream = (hipStream_t)stream;
  return OZAKI2_OK;
}

int ozaki2_set_moduli_table(int table) {
  if (table != OZAKI2_MODULI_PAPER && table != OZAKI2_MODULI_OPTIMAL) return OZAKI2_ERR_INVALID_ARG;
  g_table = table == OZAKI2_MODULI_PAPER ? kTablePaper : kTableOptimal;
  return OZAKI2_OK;
}

int ozaki2_moduli(int table, int N, int* p_out) {
  if ((table != OZAKI2_MODULI_PAPER && table != OZAKI2_MODULI_OPTIMAL) || !p_out)
    return OZAKI2_ERR_INVALID_ARG;
  if (N < 2 || N > kMaxModuli) return OZAKI2_ERR_N_RANGE;
  return moduli_of(table == OZAKI2_MODULI_PAPER ? kTablePaper : kTableOptimal, N, p_out)
             ? OZAKI2_OK
             : OZAKI2_ERR_INIT;
}

int ozaki2_debug_constants(int prec, int table, int N, double* out) {
  if ((prec != 64 && prec != 32) || !out) return OZAKI2_ERR_INVALID_ARG;
  if (table != OZAKI2_MODULI_PAPER && table != OZAKI2_MODULI_OPTIMAL) return OZAKI2_ERR_INVALID_ARG;
  int rc = check_N(N, prec);
  if (rc) return rc;
  CrtConsts cc;
  if (!build_consts(N, prec, table == OZAKI2_MODULI_PAPER ? kTablePaper : kTableOptimal, &cc))
    return OZAKI2_ERR_INIT;
  out[0] = cc.P1;
  out[1] = cc.P2;
  out[2] = cc.Pinv;
  out[3] = cc.Pprime;
  out[4] = cc.c;
  for (int l = 0; l < N; ++l) {
    out[5 + l] = cc.s1[l];
    out[5 + N + l] = cc.s2[l];
  }
  return OZAKI2_OK;
}

size_t ozaki2_workspace_bytes(int prec, int m, int n, int k, int N) {
  if ((prec != 64 && prec != 32) || m < 0 || n < 0 || k < 0 || k > kMaxK) return 0;
  if (m > kMaxDim || n > kMaxDim || check_N(N, prec) != OZAKI2_OK) return 0;
  return layout(m, n, k, N, single_row_pad(m, n, N), N).total;
}

int ozaki2_set_workspace(void* dptr, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& st = g_dev[dev];
  st.user_ws = dptr;
  st.user_bytes = dptr ? bytes : 0;
  ++st.ws_gen;
  return OZAKI2_OK;
}

int ozaki2_sync_status(void) {
  if (hipStreamSynchronize(g_stream) != hipSuccess) return OZAKI2_ERR_HIP;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  int* status = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    status = g_dev[dev].status;
  }
  // The workspace path's word and the allocation-free entry point's word.
  int any = 0;
  for (int* w : {status, noalloc_status(dev)}) {
    if (!w) continue;
    int h = 0;
    if (hipMemcpy(&h, w, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return OZAKI2_ERR_HIP;
    if (h && hipMemset(w, 0, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
    any |= h;
  }
  return any ? OZAKI2_ERR_NONFINITE : OZAKI2_OK;
}

int ozaki2_gemm_batched(int prec, int count, const int* mnkN, const void* const* A, const int* lda,
                        const void* const* B, const int* ldb, void* const* C, const int* ldc) {
  if ((prec != 64 && prec != 32) || count < 0) return OZAKI2_ERR_INVALID_ARG;
  if (count == 0) return OZAKI2_OK;
  if (!mnkN || !A || !lda || !B || !ldb || !C || !ldc) return OZAKI2_ERR_INVALID_ARG;
  return batched_impl(prec == 64 ? Prec::F64 : Prec::F32, count, mnkN, A, lda, B, ldb, C, ldc);
}

size_t ozaki2_batched_workspace_bytes(int prec, int count, const int* mnkN) {
  if ((prec != 64 && prec != 32) || count < 0 || (count > 0 && !mnkN)) return 0;
  const int nmax = prec == 64 ? kMaxModuli : 16;
  for (int p = 0; p < count; ++p) {
    const int m = mnkN[4 * p], n = mnkN[4 * p + 1], k = mnkN[4 * p + 2], N = mnkN[4 * p + 3];
    if (m < 0 || n < 0 || k < 0 || k > kMaxK || N < 2 || N > nmax) return 0;
    if (m > kMaxDim || n > kMaxDim) return 0;
  }
  return batch_layout(count, mnkN, nullptr, nullptr);
}

}  // extern "C" (reopened below)

namespace {

// The N-independent planner terms (Algorithm 2's scaling pass, row and column
// sums of the scaled |A| and |B|, the BF16 lower bound of S) into the planner
// region `ws` with layout L; enqueued on s.
void plan_terms(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                const PlanLayout& L, char* ws, hipStream_t s) {
  uint64_t* rowbits = at<uint64_t>(ws, L.rowbits);
  uint64_t* colbits = at<uint64_t>(ws, L.colbits);
  int* rmax = at<int>(ws, L.rmax);
  int* cmax = at<int>(ws, L.cmax);
  int* flag = at<int>(ws, L.flag);
  CrtConsts cc;
  std::memset(&cc, 0, sizeof(cc));
  Scope sc(PH_PLAN, s);
  launch_init(s, rowbits, L.mp, colbits, L.np, rmax, cmax, flag);
  launch_absmax_rows(s, pr, A, lda, m, k, rowbits, flag);
  // Cbar maxima exactly as the emulation computes them (Algorithm 2)
  launch_slices(s, pr, 0, true, A, lda, m, k, L.mp, L.kp, rowbits, nullptr, cc,
                at<int8_t>(ws, L.Abar));
  if (L.kp <= kAbsBarMaxK) {
    launch_absbar_cols(s, pr, B, ldb, k, n, L.np, L.kp, colbits, flag, at<int8_t>(ws, L.Bbar));
  } else {
    launch_absmax_cols(s, pr, B, ldb, k, n, colbits, flag);
    launch_slices(s, pr, 0, false, B, ldb, n, k, L.np, L.kp, colbits, nullptr, cc,
                  at<int8_t>(ws, L.Bbar));
  }
  // and one byte per entry, Cbar_ij != 0, which holds exactly when
  // (|A||B|)_ij > 0 (Abar, Bbar are >= 1 wherever A, B are nonzero): an
  // entry whose lower bound of S below underflows to 0 is then known to be
  // nonzero, and no N is accepted for it
  launch_gemm_i8(s, 3, at<int8_t>(ws, L.Abar), 0, at<int8_t>(ws, L.Bbar), 0, L.mp, L.np, L.kp, 1,
                 cc, at<int8_t>(ws, L.mask), 0, L.mp, rmax, cmax);
  // scaled |A|, |B| as BF16 lower bounds, with upward row / column sums
  launch_plan_slices(s, pr, true, A, lda, m, k, L.mp, L.kp, rowbits, at<uint16_t>(ws, L.Abf),
                     at<double>(ws, L.pr));
  launch_plan_slices(s, pr, false, B, ldb, n, k, L.np, L.kp, colbits, at<uint16_t>(ws, L.Bbf),
                     at<double>(ws, L.pc));
  launch_plan_vectors(s, at<double>(ws, L.pr), L.mp, at<double>(ws, L.pc), L.np, L.kp / 64, rmax,
                      cmax, m, n, at<double>(ws, L.rs), at<double>(ws, L.cs), at<double>(ws, L.sr),
                      at<double>(ws, L.sc));
  launch_gemm_bf16_store(s, at<uint16_t>(ws, L.Abf), at<uint16_t>(ws, L.Bbf), L.mp, L.np, L.kp,
                         at<float>(ws, L.S), L.mp);
}

// BF16 products of the truncated operands are exact in FP32; each of the k
// accumulation steps loses at most 2^-23 relative (all terms >= 0).
double bf16_acc_scale(int k) { return 1.0 - (double)k * 0x1p-22; }

// The smallest N in [2, nhi] whose N-dependent bound is within eps of S on
// every entry (reading R16), from terms that plan_terms has enqueued.
// Synchronises.  OZAKI2_ERR_UNREACHABLE (N_out = nhi) if there is none,
// OZAKI2_ERR_NONFINITE if an input entry was not finite.
int plan_search(const PlanLayout& L, char* ws, int m, int n, int k, double eps, const PlanCoef& pc,
                int nhi, hipStream_t s, int* N_out) {
  int* flag = at<int>(ws, L.flag);
  int* res = at<int>(ws, L.res);
  PlanTable pt;
  std::memset(&pt, 0, sizeof(pt));
  pt.nlo = 2;
  pt.nhi = nhi;
  pt.k = (double)k;
  pt.eps = eps;
  pt.acc_scale = bf16_acc_scale(k);
  for (int N = 2; N <= kMaxModuli; ++N) {
    pt.t[N] = pc.t[N];
    pt.tt[N] = pc.tt[N];
    pt.extra[N] = pc.extra[N];
  }
  const float* S = at<float>(ws, L.S);
  const uint8_t* mask = at<uint8_t>(ws, L.mask);
  const double *rs = at<double>(ws, L.rs), *cs = at<double>(ws, L.cs);
  const double *sr = at<double>(ws, L.sr), *scv = at<double>(ws, L.sc);
  if (hipMemsetAsync(res, 0, 2 * sizeof(int), s) != hipSuccess) return OZAKI2_ERR_HIP;
  launch_plan_entries(s, S, mask, L.mp, m, n, rs, cs, sr, scv, pt, res);
  // The largest per-entry minimum is checked on every entry in the same
  // round trip (the bound is not monotone in N once the N-dependent
  // accumulation term dominates, so it may fail somewhere).
  launch_plan_verify(s, S, mask, L.mp, m, n, rs, cs, sr, scv, pt, 0, res, res + 1);
  int host[2] = {0, 0};
  int hflag = 0;
  if (hipMemcpyAsync(host, res, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OZAKI2_ERR_HIP;
  if (hflag) {
    *N_out = nhi;
    return OZAKI2_ERR_NONFINITE;
  }
  int N = host[0] < 2 ? 2 : host[0];
  if (N <= nhi && host[1]) {
    // N failed on some entry: the smallest larger N that satisfies all.
    for (++N; N <= nhi; ++N) {
      if (hipMemsetAsync(res + 1, 0, sizeof(int), s) != hipSuccess) return OZAKI2_ERR_HIP;
      launch_plan_verify(s, S, mask, L.mp, m, n, rs, cs, sr, scv, pt, N, nullptr, res + 1);
      int bad = 0;
      if (hipMemcpyAsync(&bad, res + 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return OZAKI2_ERR_HIP;
      if (!bad) break;
    }
  }
  if (N > nhi) {
    *N_out = nhi;
    return OZAKI2_ERR_UNREACHABLE;
  }
  *N_out = N;
  return OZAKI2_OK;
}

// Workspace of the certified call at N: the planner region, then the
// single-problem layout.
size_t certified_bytes(int m, int n, int k, int N, size_t* gemm_off) {
  const size_t off = rup(plan_layout(m, n, k).total, 256);
  if (gemm_off) *gemm_off = off;
  return off + layout(m, n, k, N, single_row_pad(m, n, N), N).total;
}

}  // namespace

extern "C" {

// The planner on the real embedding of a complex product (the form of
// ozaki2_zgemm): Ahat and Bhat are written into the workspace, followed by
// the planner's own layout for the 2m x n x 2k problem.
int ozaki2_zrequired_moduli(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                            int ldb, double eps, int* N_out) {
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  if (!N_out || !(eps > 0.0) || !(eps < INFINITY)) return OZAKI2_ERR_INVALID_ARG;
  int rc = check_complex_args(m, n, k, A, lda, B, ldb, nullptr, 0, kMaxK / 2, false);
  if (rc) return rc;
  const int nhi = prec == 64 ? kMaxModuli : 16;
  if (m == 0 || n == 0 || k == 0) {  // AB = 0 is represented exactly
    *N_out = 2;
    return OZAKI2_OK;
  }
  const Prec pr = prec == 64 ? Prec::F64 : Prec::F32;
  PlanCoef pc;
  if ((rc = get_plan_coef(prec, &pc))) return rc;
  const size_t es = pr == Prec::F64 ? 8 : 4;
  const size_t Bh = rup(es * 4 * (size_t)m * k, 256);
  const size_t off = rup(Bh + es * 2 * (size_t)k * n, 256);
  const PlanLayout L = plan_layout(2 * m, n, 2 * k);
  char* ws;
  int* status;
  if ((rc = get_workspace(off + L.total, &ws, &status))) return rc;
  hipStream_t s = g_stream;
  launch_embed_complex(s, pr, A, lda, B, ldb, m, n, k, ws, ws + Bh);
  plan_terms(pr, 2 * m, n, 2 * k, ws, 2 * m, ws + Bh, 2 * k, L, ws + off, s);
  return plan_search(L, ws + off, 2 * m, n, 2 * k, eps, pc, nhi, s, N_out);
}

int ozaki2_required_moduli(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                           int ldb, double eps, int* N_out) {
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  if (!N_out || !(eps > 0.0) || !(eps < INFINITY)) return OZAKI2_ERR_INVALID_ARG;
  int rc = check_args(m, n, k, A, lda, B, ldb, nullptr, 1, false);
  if (rc) return rc;
  const int nhi = prec == 64 ? kMaxModuli : 16;
  if (m == 0 || n == 0 || k == 0) {  // AB = 0 is represented exactly
    *N_out = 2;
    return OZAKI2_OK;
  }
  const Prec pr = prec == 64 ? Prec::F64 : Prec::F32;
  PlanCoef pc;
  if ((rc = get_plan_coef(prec, &pc))) return rc;
  PlanLayout L = plan_layout(m, n, k);
  char* ws;
  int* status;
  if ((rc = get_workspace(L.total, &ws, &status))) return rc;
  hipStream_t s = g_stream;
  plan_terms(pr, m, n, k, A, lda, B, ldb, L, ws, s);
  return plan_search(L, ws, m, n, k, eps, pc, nhi, s, N_out);
}

size_t ozaki2_certified_workspace_bytes(int prec, int m, int n, int k, int N) {
  if (prec != 64 && prec != 32) return 0;
  if (m < 0 || n < 0 || k < 0 || k > kMaxK || N < 2 || N > (prec == 64 ? kMaxModuli : 16))
    return 0;
  if (m > kMaxDim || n > kMaxDim) return 0;
  if (m == 0 || n == 0 || k == 0) return 0;
  return certified_bytes(m, n, k, N, nullptr);
}

int ozaki2_gemm_certified(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                          int ldb, void* C, int ldc, double eps, int N_start, int* N_used,
                          double* ratio) {
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  if (!N_used || !(eps > 0.0) || !(eps < INFINITY)) return OZAKI2_ERR_INVALID_ARG;
  int rc = check_args(m, n, k, A, lda, B, ldb, C, ldc, true);
  if (rc) return rc;
  const int b = prec, nhi = prec == 64 ? kMaxModuli : 16;
  if (N_start != 0 && (rc = check_N(N_start, b))) return rc;
  const Prec pr = prec == 64 ? Prec::F64 : Prec::F32;
  hipStream_t s = g_stream;
  if (m == 0 || n == 0 || k == 0) {  // AB = 0 is represented exactly
    *N_used = N_start ? N_start : 2;
    if (ratio) *ratio = 0.0;
    if (m == 0 || n == 0) return OZAKI2_OK;
    launch_fill_zero(s, pr, C, ldc, m, n);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return OZAKI2_ERR_HIP;
    return OZAKI2_OK;
  }
  PlanCoef pc;
  if ((rc = get_plan_coef(prec, &pc))) return rc;
  const PlanLayout Lp = plan_layout(m, n, k);
  uint64_t terms_gen = 0;  // workspace generation the planner terms were computed in
  int N = N_start;
  for (;;) {
    const int Nw = N ? N : 2;
    size_t off;
    const size_t total = certified_bytes(m, n, k, Nw, &off);
    char* ws;
    int* status;
    uint64_t gen = 0;
    if ((rc = get_workspace(total, &ws, &status, &gen))) return rc;
    if (gen != terms_gen) {  // first pass, or the workspace moved
      plan_terms(pr, m, n, k, A, lda, B, ldb, Lp, ws, s);
      terms_gen = gen;
      if (N == 0) {
        rc = plan_search(Lp, ws, m, n, k, eps, pc, nhi, s, &N);
        // A non-finite input: one run at N = 2 writes the NaN output and
        // records the status, and the check below returns the error.
        if (rc == OZAKI2_ERR_NONFINITE) N = 2;
        else if (rc != OZAKI2_OK && rc != OZAKI2_ERR_UNREACHABLE) return rc;
        continue;  // the layout depends on N
      }
    }
    CrtConsts cc;
    if ((rc = get_consts(N, b, &cc))) return rc;
    const Layout Lg = layout(m, n, k, N, single_row_pad(m, n, N), N);
    char* wg = ws + off;
    // The planner terms include the scaling pass of Algorithm 2 on the same
    // inputs (the same kernels, so the same bits): the runs start from it.
    const PreScale pre{at<uint64_t>(ws, Lp.rowbits), at<uint64_t>(ws, Lp.colbits),
                       at<int>(ws, Lp.rmax), at<int>(ws, Lp.cmax), at<int>(ws, Lp.flag)};
    if ((rc = run_pipeline(pr, m, n, k, A, lda, B, ldb, C, ldc, cc, Lg, wg, status, s, false,
                           &pre)))
      return rc;
    CertTable ct;
    ct.t = pc.t[N];
    ct.tt = pc.tt[N];
    ct.extra = pc.extra[N];
    ct.rconst = pc.rconst[N];
    ct.rel = pc.rel[N];
    ct.k = (double)k;
    ct.acc_scale = bf16_acc_scale(k);
    ct.tiny = prec == 64 ? 0x1p-1074 : 0x1p-149;
    unsigned long long* word = at<unsigned long long>(ws, Lp.res);
    if (hipMemsetAsync(word, 0, sizeof(*word), s) != hipSuccess) return OZAKI2_ERR_HIP;
    launch_certify(s, pr, C, ldc, at<int>(wg, Lg.mu), at<int>(wg, Lg.nu), at<float>(ws, Lp.S),
                   at<uint8_t>(ws, Lp.mask), Lp.mp, m, n, at<double>(ws, Lp.rs), at<double>(ws, Lp.cs),
                   at<double>(ws, Lp.sr), at<double>(ws, Lp.sc), ct, word);
    unsigned long long bits = 0;
    int hflag = 0;
    if (hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&hflag, pre.flag, sizeof(int), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return OZAKI2_ERR_HIP;
    double r;
    std::memcpy(&r, &bits, sizeof(r));
    *N_used = N;
    if (ratio) *ratio = r;
    if (hflag) return OZAKI2_ERR_NONFINITE;
    if (r <= eps) return OZAKI2_OK;
    if (N >= nhi) return OZAKI2_ERR_UNREACHABLE;
    ++N;
  }
}

int ozaki2_debug_stages(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                        int ldb, int N, int nout, void* const* out) {
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  if (!out || nout < 10 || nout > kDebugOutputs || !out[9]) return OZAKI2_ERR_INVALID_ARG;
  void* all[kDebugOutputs] = {};
  for (int q = 0; q < nout; ++q) all[q] = out[q];
  return gemm_impl(prec == 64 ? Prec::F64 : Prec::F32, m, n, k, A, lda, B, ldb, out[9],
                   m > 1 ? m : 1, N, all);
}

int ozaki2_debug_mfma_probe(int iters, int changing, float* ms, double* ops) {
  if (iters < 1 || iters > (1 << 20) || !ms || !ops) return OZAKI2_ERR_INVALID_ARG;
  if (changing != 0 && changing != 1) return OZAKI2_ERR_INVALID_ARG;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return OZAKI2_ERR_HIP;
  return probe_mfma(g_stream, cus, iters, changing != 0, ms, ops);
}

int ozaki2_debug_log2f(const float* d, float* out, int count) {
  if (count < 0 || (count > 0 && (!d || !out))) return OZAKI2_ERR_INVALID_ARG;
  if (count == 0) return OZAKI2_OK;
  launch_log2f(g_stream, d, out, count);
  return hipGetLastError() == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
}

int ozaki2_profile(int enable) {
  for (auto& r : g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  g_prof = enable != 0;
  return OZAKI2_OK;
}

int ozaki2_profile_read(int* phase, float* ms, int cap) {
  if (hipStreamSynchronize(g_stream) != hipSuccess) return OZAKI2_ERR_HIP;
  int n = 0;
  for (auto& r : g_recs) {
    if (n >= cap) break;
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return OZAKI2_ERR_HIP;
    if (phase) phase[n] = r.phase;
    if (ms) ms[n] = t;
    ++n;
  }
  return n;
}

const char* ozaki2_profile_name(int phase) {
  return (phase >= 0 && phase < PH_COUNT) ? kPhaseNames[phase] : "";
}

int ozaki2_debug_tuning(int knob, int value, int* previous) {
  std::atomic<int>* k = nullptr;
  switch (knob) {
    case OZAKI2_KNOB_SLICE_WORKGROUPS:
      if (value < 0) return OZAKI2_ERR_INVALID_ARG;
      k = &g_slice_cap;
      break;
    case OZAKI2_KNOB_GEMM_TILE:
      if (value < 0 || value > 2) return OZAKI2_ERR_INVALID_ARG;
      k = &g_gemm_tile;
      break;
    case OZAKI2_KNOB_BATCH_SPLIT:
      if (value < -1) return OZAKI2_ERR_INVALID_ARG;
      k = &g_batch_split;
      break;
    case OZAKI2_KNOB_BATCH_GRAPH:
      if (value != 0 && value != 1) return OZAKI2_ERR_INVALID_ARG;
      k = &g_batch_graph;
      break;
    case OZAKI2_KNOB_BATCH_PERSIST:
      if (value < -1 || value > 2) return OZAKI2_ERR_INVALID_ARG;
      k = &g_batch_persist;
      break;
    case OZAKI2_KNOB_SPLIT_K:
      if (value != 0 && value != 1) return OZAKI2_ERR_INVALID_ARG;
      k = &g_split_k;
      break;
    default:
      return OZAKI2_ERR_INVALID_ARG;
  }
  const int old = k->exchange(value);
  if (previous) *previous = old;
  return OZAKI2_OK;
}

const char* ozaki2_version(void) { return "ozaki2-gfx950 0.2"; }

}  // extern "C"
