// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the round function and
// the ten-round bijection of a 128-bit counter under a 64-bit key, for the
// device code that draws the method's random numbers (Gaussian test matrices,
// the signs and column subset of the structured sketch).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  uint32_t hi0 = __umulhi(m0, c0), lo0 = m0 * c0;
  uint32_t hi1 = __umulhi(m1, c2), lo1 = m1 * c2;
  uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
  c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
}

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  philox_round(c[0], c[1], c[2], c[3], k0, k1);
#pragma unroll
  for (int r = 1; r < 10; ++r) {
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    philox_round(c[0], c[1], c[2], c[3], k0, k1);
  }
}

}  // namespace rsvd
