// C ABI of the Ozaki-II emulated GEMM (include/ozaki2.h): argument checks,
// workspace management, constant-table cache and the launch sequence of
// Algorithm 1 (Scaling -> CRT -> inverse scaling) on one HIP stream.
#include "../../include/ozaki2.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "ozaki2_internal.h"

using namespace oz2;

namespace {

thread_local hipStream_t g_stream = nullptr;

struct DeviceState {
  void* ws = nullptr;          // library-owned workspace
  size_t ws_bytes = 0;
  void* user_ws = nullptr;     // caller-installed workspace (takes precedence)
  size_t user_bytes = 0;
  int* status = nullptr;       // sticky data-dependent status word
};
std::mutex g_mu;
std::map<int, DeviceState> g_dev;
std::map<int, CrtConsts> g_consts;  // key: N * 100 + b

// ---------------------------------------------------------------------------
// profiling (HIP events around each phase on the library stream)
// ---------------------------------------------------------------------------
enum Phase {
  PH_INIT, PH_ABSMAX_A, PH_ABSMAX_B, PH_BAR_A, PH_BAR_B, PH_GEMM_SCALE, PH_SHIFTS, PH_RES_A,
  PH_RES_B, PH_GEMM_RES, PH_CRT, PH_PLAN, PH_COUNT
};
const char* kPhaseNames[PH_COUNT] = {"init", "absmax_A", "absmax_B", "bar_A", "bar_B",
                                     "gemm_scale", "shifts", "residue_A", "residue_B",
                                     "gemm_residue", "crt", "plan"};
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
  size_t rowbits, colbits, rmax, cmax, mu_p, nu_p, mu, nu, ef, flag, A, B, W, total;
};

Layout layout(int m, int n, int k, int N) {
  Layout L;
  L.mp = (int)rup((size_t)(m > 0 ? m : 1), kRowPad);
  L.np = (int)rup((size_t)(n > 0 ? n : 1), kRowPad);
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
  L.ef = take(4ull * (L.mp + L.np));
  L.flag = take(4);
  L.A = take((size_t)N * L.mp * L.kp);
  L.B = take((size_t)N * L.np * L.kp);
  L.W = take((size_t)N * L.np * L.mp);
  L.total = off;
  return L;
}

int check_args(int m, int n, int k, const void* A, int lda, const void* B, int ldb, const void* C,
               int ldc, bool needC) {
  if (m < 0 || n < 0 || k < 0) return OZAKI2_ERR_INVALID_ARG;
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

int get_consts(int N, int b, CrtConsts* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  int key = N * 100 + b;
  auto it = g_consts.find(key);
  if (it == g_consts.end()) {
    CrtConsts cc;
    if (!build_consts(N, b, &cc)) return OZAKI2_ERR_INIT;
    it = g_consts.emplace(key, cc).first;
  }
  *out = it->second;
  return OZAKI2_OK;
}

// Returns a device workspace of at least `bytes` for the current device.
int get_workspace(size_t bytes, char** base, int** status) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& st = g_dev[dev];
  if (!st.status) {
    if (hipMalloc(&st.status, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
    if (hipMemset(st.status, 0, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
  }
  *status = st.status;
  if (st.user_ws) {
    if (st.user_bytes < bytes) return OZAKI2_ERR_WORKSPACE;
    *base = (char*)st.user_ws;
    return OZAKI2_OK;
  }
  if (st.ws_bytes < bytes) {
    if (st.ws) {
      if (hipDeviceSynchronize() != hipSuccess) return OZAKI2_ERR_HIP;
      (void)hipFree(st.ws);
      st.ws = nullptr;
      st.ws_bytes = 0;
    }
    if (hipMalloc(&st.ws, bytes) != hipSuccess) return OZAKI2_ERR_HIP;
    st.ws_bytes = bytes;
  }
  *base = (char*)st.ws;
  return OZAKI2_OK;
}

template <typename P>
P* at(char* base, size_t off) {
  return reinterpret_cast<P*>(base + off);
}

// The launch sequence of Algorithm 1 for one problem (m, n, k >= 1).
int run_pipeline(Prec pr, int m, int n, int k, const void* A, int lda, const void* B, int ldb,
                 void* C, int ldc, const CrtConsts& cc, const Layout& L, char* ws, int* status,
                 hipStream_t s, bool want_ef) {
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
  {
    Scope sc(PH_INIT, s);
    launch_init(s, rowbits, L.mp, colbits, L.np, rmax, cmax, flag);
  }
  {
    Scope sc(PH_ABSMAX_A, s);
    launch_absmax_rows(s, pr, A, lda, m, k, rowbits, flag);
  }
  {
    Scope sc(PH_ABSMAX_B, s);
    launch_absmax_cols(s, pr, B, ldb, k, n, colbits, flag);
  }
  // Abar = ceil(2^mu' |A|), Bbar = ceil(|B| 2^nu') into slice 0 of the operand buffers.
  {
    Scope sc(PH_BAR_A, s);
    launch_slices(s, pr, 0, true, A, lda, m, k, L.mp, L.kp, rowbits, nullptr, cc, As);
  }
  {
    Scope sc(PH_BAR_B, s);
    launch_slices(s, pr, 0, false, B, ldb, n, k, L.np, L.kp, colbits, nullptr, cc, Bs);
  }
  // Cbar = Abar Bbar; keep row maxima (over j) and column maxima (over i).
  {
    Scope sc(PH_GEMM_SCALE, s);
    launch_gemm_i8(s, 1, As, 0, Bs, 0, L.mp, L.np, L.kp, 1, cc, nullptr, 0, 0, rmax, cmax);
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
                   cc.N, cc, W, (size_t)L.np * L.mp, L.mp, nullptr, nullptr);
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
  Layout L = layout(m, n, k, N);
  char* ws;
  int* status;
  if ((rc = get_workspace(L.total, &ws, &status))) return rc;
  rc = run_pipeline(pr, m, n, k, A, lda, B, ldb, C, ldc, cc, L, ws, status, s, dbg != nullptr);
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
  return hipStreamSynchronize(s) == hipSuccess ? OZAKI2_OK : OZAKI2_ERR_HIP;
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

int ozaki2_set_stream(void* stream) {
  g_stream = (hipStream_t)stream;
  return OZAKI2_OK;
}

size_t ozaki2_workspace_bytes(int prec, int m, int n, int k, int N) {
  if ((prec != 64 && prec != 32) || m < 0 || n < 0 || k < 0 || N < 2 || N > kMaxModuli) return 0;
  return layout(m, n, k, N).total;
}

int ozaki2_set_workspace(void* dptr, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& st = g_dev[dev];
  st.user_ws = dptr;
  st.user_bytes = dptr ? bytes : 0;
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
  if (!status) return OZAKI2_OK;
  int h = 0;
  if (hipMemcpy(&h, status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return OZAKI2_ERR_HIP;
  if (hipMemset(status, 0, sizeof(int)) != hipSuccess) return OZAKI2_ERR_HIP;
  return h ? OZAKI2_ERR_NONFINITE : OZAKI2_OK;
}

int ozaki2_gemm_batched(int prec, int count, const int* mnkN, const void* const* A, const int* lda,
                        const void* const* B, const int* ldb, void* const* C, const int* ldc) {
  if ((prec != 64 && prec != 32) || count < 0) return OZAKI2_ERR_INVALID_ARG;
  if (count == 0) return OZAKI2_OK;
  if (!mnkN || !A || !lda || !B || !ldb || !C || !ldc) return OZAKI2_ERR_INVALID_ARG;
  const int b = prec;
  for (int p = 0; p < count; ++p) {
    int rc = check_args(mnkN[4 * p], mnkN[4 * p + 1], mnkN[4 * p + 2], A[p], lda[p], B[p], ldb[p],
                        C[p], ldc[p], true);
    if (rc) return rc;
    if ((rc = check_N(mnkN[4 * p + 3], b))) return rc;
  }
  const Prec pr = prec == 64 ? Prec::F64 : Prec::F32;
  for (int p = 0; p < count; ++p) {
    int rc = gemm_impl(pr, mnkN[4 * p], mnkN[4 * p + 1], mnkN[4 * p + 2], A[p], lda[p], B[p],
                       ldb[p], C[p], ldc[p], mnkN[4 * p + 3], nullptr);
    if (rc) return rc;
  }
  return OZAKI2_OK;
}

int ozaki2_required_moduli(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                           int ldb, double eps, int* N_out);  // planner.cpp

int ozaki2_debug_stages(int prec, int m, int n, int k, const void* A, int lda, const void* B,
                        int ldb, int N, void* const* out) {
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  if (!out || !out[9]) return OZAKI2_ERR_INVALID_ARG;
  return gemm_impl(prec == 64 ? Prec::F64 : Prec::F32, m, n, k, A, lda, B, ldb, out[9],
                   m > 1 ? m : 1, N, out);
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

const char* ozaki2_version(void) { return "ozaki2-gfx950 0.1"; }

}  // extern "C"
