// Device helpers for the byte-wise residue kernels (complex 3-product form,
// split-k reduction).  Include from .hip sources only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ozaki2_internal.h"

namespace oz2 {

// mod(x, p) in the symmetric INT8 range of Section 1.2 ([-(p-1)/2, (p-1)/2]
// for odd p, [-128, 127] for p = 256: [hi + 1 - p, hi] with hi = (p - 1) / 2)
// for |x| < 2^14.  The FP32 quotient x (1/p) is within 2^-9 of x/p there, so
// its rounding is within one of the nearest integer to x/p, and one
// correction either way lands r in the range (checked exhaustively for every
// p <= 256 and |x| < 2^14).
__device__ inline int mod_small(int x, int p, float pinv, int hi) {
  int r = x - (int)rintf((float)x * pinv) * p;
  r -= r > hi ? p : 0;
  r += r < hi + 1 - p ? p : 0;
  return r;
}

// Signed byte i of a 32-bit word.
__device__ inline int sbyte(uint32_t w, int i) { return (int)(w << (24 - 8 * i)) >> 24; }

// mod_small for modulus l of a constant table, placed as byte i of a word.
struct SmallMod {
  int p, hi;
  float pinv;
  __device__ explicit SmallMod(const CrtConsts& cc, int l)
      : p(cc.p[l]), hi((cc.p[l] - 1) / 2), pinv((float)cc.pinv[l]) {}
  __device__ uint32_t byte(int x, int i) const {
    return (uint32_t)(mod_small(x, p, pinv, hi) & 0xFF) << (8 * i);
  }
};

}  // namespace oz2
