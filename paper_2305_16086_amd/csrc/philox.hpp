// Philox4x32-10 counter-based generator for the walk kernels.
//
// Written from the published definition (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of
//   (x0,x1,x2,x3) -> (hi(B*x2) ^ x1 ^ k0, lo(B*x2), hi(A*x0) ^ x3 ^ k1, lo(A*x0))
// with A = 0xD2511F53, B = 0xCD9E8D57, the key advancing by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sc {

struct U32x4 {
  uint32_t w[4];
};

__host__ __device__ inline void philox_mul(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  const uint64_t p = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
  hi = static_cast<uint32_t>(p >> 32);
  lo = static_cast<uint32_t>(p);
}

__host__ __device__ inline U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kA = 0xD2511F53u, kB = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hA, lA, hB, lB;
    philox_mul(kA, c0, hA, lA);
    philox_mul(kB, c2, hB, lB);
    const uint32_t n0 = hB ^ c1 ^ k0;
    const uint32_t n2 = hA ^ c3 ^ k1;
    c0 = n0;
    c1 = lB;
    c2 = n2;
    c3 = lA;
    k0 += kW0;
    k1 += kW1;
  }
  U32x4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

// Neighbour position in [0, d): floor(word * d / 2^32).
__host__ __device__ inline uint32_t pick_neighbour(uint32_t word, uint32_t d) {
  return static_cast<uint32_t>((static_cast<uint64_t>(word) * d) >> 32);
}

}  // namespace sc
