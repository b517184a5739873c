// Allocation-free single-problem entry point (ozaki2_gemm_noalloc): the same
// launch sequence as ozaki2_gemm / ozaki2_sgemm, with its workspace in a
// fixed-size device array instead of memory from hipMalloc, for callers
// that cannot allocate.
//
// `scratch` is a device variable: in host code its name is only a host-side
// stand-in.  Each device holds its own copy at its own address, which
// hipGetSymbolAddress returns with that device current; that address, kept
// per device, is what every kernel receives.  The first 256 bytes hold the
// sticky status word (zero when the code object is loaded, cleared by
// ozaki2_sync_status after it reports); the workspace follows.  Every
// per-call field of the workspace (abs-max bit patterns, maxima of Cbar,
// the non-finite flag) is set by the call's own init kernel, so nothing
// else needs clearing between calls.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "../../include/ozaki2.h"
#include "ozaki2_internal.h"

namespace oz2 {
namespace {

constexpr size_t kScratchBytes = OZAKI2_NOALLOC_SCRATCH_BYTES;
constexpr size_t kStatusBytes = 256;   // status word, then the workspace
static_assert(kScratchBytes % 256 == 0 && kScratchBytes > kStatusBytes, "scratch size");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDev = 64;
std::atomic<char*> g_scratch[kMaxDev];
std::mutex g_setup_mu;

// This device's copy of `scratch`, set up on the first call on the device:
// the device address of the array, and the slice kernels' launch figures
// that the workspace path also sets up per device.
int scratch_on_device(char** ws, int** status) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZAKI2_ERR_HIP;
  if (dev < 0 || dev >= kMaxDev) return OZAKI2_ERR_HIP;
  char* base = g_scratch[dev].load(std::memory_order_acquire);
  if (!base) {
    std::lock_guard<std::mutex> lk(g_setup_mu);
    base = g_scratch[dev].load(std::memory_order_relaxed);
    if (!base) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return OZAKI2_ERR_HIP;
      init_slice_launch(dev);
      base = static_cast<char*>(ptr);
      g_scratch[dev].store(base, std::memory_order_release);
    }
  }
  *status = reinterpret_cast<int*>(base);
  *ws = base + kStatusBytes;
  return OZAKI2_OK;
}

}  // namespace

int* noalloc_status(int dev) {
  if (dev < 0 || dev >= kMaxDev) return nullptr;
  return reinterpret_cast<int*>(g_scratch[dev].load(std::memory_order_acquire));
}

}  // namespace oz2

extern "C" int ozaki2_gemm_noalloc(int prec, int m, int n, int k, const void* A, int lda,
                                   const void* B, int ldb, void* C, int ldc, int N) {
  using namespace oz2;
  if (prec != 64 && prec != 32) return OZAKI2_ERR_INVALID_ARG;
  return gemm_on_buffer(prec == 64 ? Prec::F64 : Prec::F32, m, n, k, A, lda, B, ldb, C, ldc, N,
                        kScratchBytes - kStatusBytes, scratch_on_device);
}
