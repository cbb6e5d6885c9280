// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// from its published definition: 10 rounds of two 32x32->64 multiplications
// with the round constants 0xD2511F53, 0xCD9E8D57 and the Weyl key increments
// 0x9E3779B9, 0xBB67AE85.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nqs {

__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                     uint32_t out[4]) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

}  // namespace nqs
