// philox.h -- Philox4x32-10 counter-based generator for device code
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC'11): ten rounds of two 32x32->64 multiplies by the round
// multipliers and xors with the key, which is bumped by the two Weyl
// constants between rounds.  Only word 0 of the output is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tr {

__device__ __forceinline__ uint32_t philox4x32_10_w0(uint32_t c0, uint32_t c1,
                                                     uint32_t c2, uint32_t c3,
                                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c0;
}

// The simulation's draw: counter (vehicle id, t, sub-step, 0).
__device__ __forceinline__ uint32_t veh_draw(uint32_t id, uint32_t t,
                                             uint32_t substep, uint32_t k0,
                                             uint32_t k1) {
  return philox4x32_10_w0(id, t, substep, 0u, k0, k1);
}

}  // namespace tr
