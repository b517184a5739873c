// MFMA-rate probe: v_mfma_i32_32x32x32_i8, the instruction of the residue
// products, issued back to back on INT8 operands that change every step,
// with no memory traffic at all.  The rate it sustains is the ceiling the
// chip's power limit leaves for that instruction on changing data, against
// which the residue products can be read (a measurement aid, not part of
// the method).
//
// Each workgroup is 8 waves, each wave 2 x 4 accumulators of 32 x 32 (the
// shape of one wave's 64 x 128 share of a 256 x 256 residue-product tile),
// one workgroup per CU as in the product kernel.  Per step a wave issues 8
// MFMAs; with CHANGE it also adds an odd constant to each of its 24 operand
// dwords (a Weyl sequence per dword, so every byte keeps changing), without
// it the operands stay fixed (the issue rate with little data toggling).
// Each thread stores one checksum word at the end so that no MFMA can be
// dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ozaki2.h"
#include "ozaki2_internal.h"

namespace oz2 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kProbeThreads = 512;
constexpr int kProbeMaxBlocks = 1024;
__device__ int g_probe_sink[kProbeMaxBlocks * kProbeThreads];

template <bool CHANGE>
__global__ __launch_bounds__(kProbeThreads, 1) void k_mfma_probe(int iters, int* __restrict__ sink) {
  const int t = blockIdx.x * kProbeThreads + threadIdx.x;
  uint32_t h = (uint32_t)t * 2654435761u + 0x6a09e667u;
  auto next = [&h]() {
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return (int)h;
  };
  v4i a[2], b[4];
#pragma unroll
  for (int i = 0; i < 2; ++i) a[i] = v4i{next(), next(), next(), next()};
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = v4i{next(), next(), next(), next()};
  v16i acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    if constexpr (CHANGE) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] += v4i{(int)0x9e3779b9, (int)0x7f4a7c15, (int)0x85ebca6b, (int)0xc2b2ae35};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] += v4i{(int)0x27d4eb2f, (int)0x165667b1, (int)0xd3a2646c, (int)0xfd7046c5};
    }
  }
  int x = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) x ^= acc[i][j][r];
  sink[t] = x;
}

}  // namespace

int probe_mfma(hipStream_t s, int blocks, int iters, bool change, float* ms, double* ops) {
  if (blocks < 1 || blocks > kProbeMaxBlocks || iters < 1) return OZAKI2_ERR_INVALID_ARG;
  int* sink = nullptr;
  if (hipGetSymbolAddress((void**)&sink, HIP_SYMBOL(g_probe_sink)) != hipSuccess)
    return OZAKI2_ERR_HIP;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return OZAKI2_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return OZAKI2_ERR_HIP;
  }
  (void)hipEventRecord(e0, s);
  if (change)
    hipLaunchKernelGGL(k_mfma_probe<true>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s, iters,
                       sink);
  else
    hipLaunchKernelGGL(k_mfma_probe<false>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s, iters,
                       sink);
  (void)hipEventRecord(e1, s);
  float t = 0.0f;
  const bool ok = hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                  hipEventElapsedTime(&t, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return OZAKI2_ERR_HIP;
  *ms = t;
  // 8 MFMAs of 2 x 32 x 32 x 32 operations per wave and step
  *ops = (double)blocks * (kProbeThreads / 64) * (double)iters * 8.0 * 65536.0;
  return OZAKI2_OK;
}

}  // namespace oz2
