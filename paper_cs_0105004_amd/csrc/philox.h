// philox.h -- Philox4x32-10 counter-based generator for device code
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC'11): ten rounds of two 32x32->64 multiplies by the round
// multipliers and xors with the key, which is bumped by the two Weyl
// constants between rounds.  Only word 0 of the output is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tr {

// One 32x32->64 multiply as a single v_mad_u64_u32 (the compiler otherwise
// issues a mul_lo/mul_hi pair for it).
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t m) {
  uint64_t r;
  asm("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(a), "s"(m) : "vcc");
  return r;
}

__device__ __forceinline__ uint32_t philox4x32_10_w0(uint32_t c0, uint32_t c1,
                                                     uint32_t c2, uint32_t c3,
                                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = mul_wide(c0, 0xD2511F53u);
    const uint64_t p1 = mul_wide(c2, 0xCD9E8D57u);
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
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
