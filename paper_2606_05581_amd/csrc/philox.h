// Walk randomness shared by the walk kernels of the library: the
// counter-based Philox4x32-10 generator and the map of its words to
// uniforms. Every random number of a walk is one word of the block for the
// counter (row, walk, step, purpose << 24 | mesh) under the key (seed lo,
// seed hi).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msk {

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon et al. (SC 2011): ten rounds of two
// 32x32->64-bit multiplies with Weyl-sequence round keys.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Top 23 bits -> centre of one of 2^23 cells of (0,1); exact in binary32.
__device__ __forceinline__ float unit_f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * (1.0f / 8388608.0f); }

enum : uint32_t { kPurposeStep = 0, kPurposeHatStart = 1, kPurposeSplit = 2, kPurposeReentry = 3, kPurposeBall = 4 };

}  // namespace msk
