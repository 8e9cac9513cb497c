// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11)
// on the device: a 4-word counter and a 2-word key; each of the 10 rounds
// multiplies words 0 and 2 by two constants and mixes the 128-bit products'
// halves with words 1 and 3 and the round key, which is bumped by two Weyl
// constants between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace ppcg {

struct U64x4 {
  uint64_t x0, x1, x2, x3;
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c.x0), lo0 = M0 * c.x0;
    const uint64_t hi1 = __umul64hi(M1, c.x2), lo1 = M1 * c.x2;
    c = U64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
  }
  return c;
}

}  // namespace ppcg
