// philox_dev.h -- counter-based random streams on the GPU.
//
// Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw (SC'11): each of
// the ten rounds multiplies counter words 0 and 2 by two fixed odd constants,
// and builds the next counter from the low halves and from the high halves
// xored with words 1 and 3 and the round key; the key is advanced by two Weyl
// increments between rounds.  The method's draws use the counter
// {draw index, cell or particle id, step, stream tag} and the seed as key.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

struct Words4 {
  uint32_t w[4];
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hiA = __umulhi(kMulA, c0), loA = kMulA * c0;
    const uint32_t hiB = __umulhi(kMulB, c2), loB = kMulB * c2;
    const uint32_t n0 = hiB ^ c1 ^ k0;
    const uint32_t n2 = hiA ^ c3 ^ k1;
    c0 = n0;
    c1 = loB;
    c2 = n2;
    c3 = loA;
    k0 += kWeylA;
    k1 += kWeylB;
  }
  Words4 out;
  out.w[0] = c0;
  out.w[1] = c1;
  out.w[2] = c2;
  out.w[3] = c3;
  return out;
}

// Word -> number conversions (each exact in double).
__device__ __forceinline__ double u24_of(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }
__device__ __forceinline__ double u53_of(uint32_t hi, uint32_t lo) {
  return (double)(((uint64_t)hi << 21) | (uint64_t)(lo >> 11)) * 0x1p-53;
}
__device__ __forceinline__ double u53_open_of(uint32_t hi, uint32_t lo) {
  const uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
  return (double)(2 * m + 1) * 0x1p-53;
}
__device__ __forceinline__ double u32_open_of(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

constexpr double kTwoPi = 6.283185307179586;

}  // namespace mpc
