// device.h -- device-side helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

namespace tr {

// Pointers read from a descriptor are generic; casting them to the global
// address space lets the compiler use global (not flat) memory instructions,
// whose completion is tracked apart from LDS traffic.
// HIP's vector classes cannot be copied out of that address space, so the
// kernels use the compiler's own vector types there.
#define GAS __attribute__((address_space(1)))
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ GAS T* gp(T* p) {
  return (GAS T*)p;
}
template <class V, class T>
__device__ __forceinline__ GAS V* gpv(T* p) {
  return (GAS V*)(void*)p;
}

__device__ __forceinline__ int wrapi(int a, int cap) {
  return a >= cap ? a - cap : a;
}

// record slot of the j-th vehicle (0 = lead) of a lane with queue word hc
__device__ __forceinline__ int rec_slot(int base, int hc, int len, int j) {
  return base + hc_par(hc) * len + wrapi(hc_head(hc) + j, len);
}

// Is the fixed-time signal at the end of the lane's link red in step t?
// (a virtual vehicle of speed zero then stands beyond the last cell)
__device__ __forceinline__ bool sig_red(const int4* s_plans, uint32_t meta,
                                        int t) {
  const int pl = lmeta_plan(meta);
  if (pl < 0) return false;
  const int4 q = s_plans[pl];
  return (int)(((uint32_t)t + (uint32_t)q.z) % (uint32_t)q.x) < q.y;
}

// The scenario's signal plans into LDS (thread j takes plan j); the caller
// orders the writes before their first use.
__device__ __forceinline__ void load_plans(const DevScen& S, int4* s_plans) {
  const int i = threadIdx.x;
  if (i < S.n_plans) s_plans[i] = S.plans[i];
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Orders this lane's LDS accesses before the next ones of any lane of the
// wavefront: a wavefront executes its LDS instructions in order, so keeping
// the compiler from moving them is enough, and nothing waits on memory.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kGroup = 2;  // chunks of 64 vehicles loaded before updating

}  // namespace tr
