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

// Wave-wide scans and reductions by DPP (data-parallel primitives): shifts
// within each row of 16 lanes, then broadcasts of lanes 15 and 31 into the
// rows above them.  Each step is one vector ALU instruction, where a
// shuffle is a round trip through the LDS crossbar.  Every lane of the
// wavefront must be active.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114,
              kDppRowShr8 = 0x118, kDppWaveShr1 = 0x138,
              kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// One step of a scan: x combined with the copy of x that the DPP control
// kCtrl moves into this lane, in the rows of kRows (a lane with no source
// row or lane combines with the identity).
template <int kCtrl, int kRows>
__device__ __forceinline__ int dpp_add(int x) {
  return x + __builtin_amdgcn_update_dpp(0, x, kCtrl, kRows, 0xf, false);
}
template <int kCtrl, int kRows>
__device__ __forceinline__ int dpp_min(int x) {
  return min(x, __builtin_amdgcn_update_dpp(INT32_MAX, x, kCtrl, kRows, 0xf,
                                            false));
}

// Inclusive prefix sum: lane i gets the sum over lanes 0..i (the wave's
// total below 2^31).
__device__ __forceinline__ int wave_scan(int x) {
  x = dpp_add<kDppRowShr1, 0xf>(x);
  x = dpp_add<kDppRowShr2, 0xf>(x);
  x = dpp_add<kDppRowShr4, 0xf>(x);
  x = dpp_add<kDppRowShr8, 0xf>(x);
  x = dpp_add<kDppRowBcast15, 0xa>(x);
  return dpp_add<kDppRowBcast31, 0xc>(x);
}

// Sum over the wavefront of values whose total is below 2^31 (every count
// the kernels sum per wavefront: vehicles, speeds, cells of a tile), as
// the 64-bit type of the counters it is added to.
__device__ __forceinline__ unsigned long long wave_sum(int v) {
  return (unsigned long long)(unsigned)__builtin_amdgcn_readlane(
      wave_scan(v), kWave - 1);
}

// Minimum over the wavefront, in a scalar register.
__device__ __forceinline__ int wave_min(int x) {
  x = dpp_min<kDppRowShr1, 0xf>(x);
  x = dpp_min<kDppRowShr2, 0xf>(x);
  x = dpp_min<kDppRowShr4, 0xf>(x);
  x = dpp_min<kDppRowShr8, 0xf>(x);
  x = dpp_min<kDppRowBcast15, 0xa>(x);
  x = dpp_min<kDppRowBcast31, 0xc>(x);
  return __builtin_amdgcn_readlane(x, kWave - 1);
}

// Lane i gets lane i - 1's x; lane 0 gets fill.
__device__ __forceinline__ int wave_prev(int x, int fill) {
  return __builtin_amdgcn_update_dpp(fill, x, kDppWaveShr1, 0xf, 0xf, false);
}

// Lane of vehicle f in a wavefront's numbering of its tile's vehicles
// (lanes in order, the vehicles of a lane consecutive): the largest lane j
// whose first vehicle vp_j is at most f, where lane thread j < nl holds
// vp_j in vp.  F and Fl are the same in every thread and bound the
// wavefront's vehicles, F <= f <= Fl < F + kWave.  Two ballots give the
// lanes of vehicles F and Fl; each thread then counts the lanes between
// them that start at or below f, reading the lane threads' registers, so
// no memory is touched.  Called by the whole wavefront.
__device__ __forceinline__ int wave_lane_of(int vp, int nl, int F, int Fl,
                                            int f) {
  const bool lt = (int)threadIdx.x < nl;
  const int l0 = __popcll(__ballot(lt && vp <= F)) - 1;
  const int l1 = __popcll(__ballot(lt && vp <= Fl)) - 1;
  int l = l0;
  for (int j = l0 + 1; j <= l1; ++j)
    l += __builtin_amdgcn_readlane(vp, j) <= f ? 1 : 0;
  return l;
}

// The value of the wavefront's last lane, in a scalar register
__device__ __forceinline__ int wave_last(int x) {
  return __builtin_amdgcn_readlane(x, kWave - 1);
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
