// ring_stats.hip -- ring-road mode (every step of a ring in one launch),
// the step counter, statistics and state export (gfx950).
#include "device.h"
#include "kernels.h"
#include "philox.h"
#include "transims.h"

namespace tr {

namespace {
constexpr int kRingBlock = 256;
}  // namespace

__global__ void k_advance(DevScen* descs, const int* slots, int n, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) descs[slots[i]].t += k;
}

// Ring mode: one workgroup holds a whole ring in LDS and runs every step.
// Vehicles are kept in cyclic order; vehicle j follows vehicle j+1 (mod n).
__global__ __launch_bounds__(kRingBlock) void k_ring(DevScen* descs,
                                                     const int* slots,
                                                     int n_steps) {
  __shared__ int sx[2][kRingMax];
  __shared__ unsigned char sv[2][kRingMax];
  __shared__ int sid[kRingMax];
  __shared__ unsigned long long s_sum;
  DevScen& S = descs[slots[blockIdx.x]];
  const int n = S.ring_n, L = S.ring_L, vmax = S.vmax;
  const int t0 = S.t;
  const int tid = threadIdx.x;
  if (tid == 0) s_sum = 0;
  for (int j = tid; j < n; j += kRingBlock) {
    sx[0][j] = S.ring_x[j];
    sv[0][j] = (unsigned char)S.ring_v[j];
    sid[j] = S.ring_id[j];
  }
  __syncthreads();
  int cur = 0;
  unsigned long long sumv = 0;
  for (int s = 0; s < n_steps; ++s) {
    const uint32_t t = (uint32_t)(t0 + s);
    for (int j = tid; j < n; j += kRingBlock) {
      const int x = sx[cur][j];
      int gap;
      if (n == 1) {
        gap = L - 1;
      } else {
        gap = sx[cur][j + 1 == n ? 0 : j + 1] - x - 1;
        if (gap < 0) gap += L;
      }
      const int v1 = min((int)sv[cur][j] + 1, vmax);
      const int v2 = min(v1, gap);
      const uint32_t u = veh_draw((uint32_t)sid[j], t, 1u, S.key0, S.key1);
      const int v3 = (v2 > 0 && (uint64_t)u < S.slow_thr) ? v2 - 1 : v2;
      int nx = x + v3;
      if (nx >= L) nx -= L;
      sx[cur ^ 1][j] = nx;
      sv[cur ^ 1][j] = (unsigned char)v3;
      sumv += v3;
    }
    cur ^= 1;
    __syncthreads();
  }
  for (int j = tid; j < n; j += kRingBlock) {
    S.ring_x[j] = sx[cur][j];
    S.ring_v[j] = sv[cur][j];
  }
  atomicAdd(&s_sum, sumv);
  __syncthreads();
  if (tid == 0) {
    S.ring_ctr[C_UPDATES] += (long long)n * n_steps;
    S.ring_ctr[C_SUMV] += (long long)s_sum;
    S.ring_ctr[C_COCC] += n > 0 ? (long long)L * n_steps : 0;
    S.t = t0 + n_steps;
  }
}

// ---- stats and state export ----------------------------------------------

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// hash of one vehicle's state (sum over vehicles = the state hash)
__device__ __forceinline__ uint64_t veh_hash(int id, int st, int link, int lane,
                                             int x, int v, int rptr) {
  const uint64_t w = (uint64_t)st | ((uint64_t)(uint32_t)lane << 4) |
                     ((uint64_t)(uint32_t)v << 8) |
                     ((uint64_t)((uint32_t)x & 0xFFFFu) << 16) |
                     ((uint64_t)(uint32_t)link << 32);
  const uint64_t h = mix64(mix64((uint64_t)(uint32_t)id) ^ w);
  return mix64(h ^ (uint64_t)(uint32_t)rptr);
}

constexpr int kWaiting = 0, kActive = 1, kArrived = 2;

}  // namespace

__global__ void k_stats(const DevScen* d, unsigned long long* out, int ring) {
  const DevScen& S = *d;
  unsigned long long h = 0, act = 0, wait = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long g0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (ring) {
    for (long long j = g0; j < S.ring_n; j += stride)
      h += veh_hash(S.ring_id[j], kActive, 0, 0, S.ring_x[j], S.ring_v[j], 0);
    act = 0;
    if (g0 == 0) {
      act = (unsigned long long)S.ring_n;
      for (int c = 0; c < C_N; ++c)
        atomicAdd(&out[c], (unsigned long long)S.ring_ctr[c]);
    }
  } else {
    // move-tile counters: one per lane at most (balanced tiles included)
    const long long n1 = S.n_veh, n2 = n1 + S.n_lanes, n3 = n2 + S.n_lanes,
                    n4 = n3 + S.n_lanes, n5 = n4 + S.n_ftiles;
    for (long long g = g0; g < n5; g += stride) {
      if (g < n1) {
        h += veh_hash((int)g, kArrived, 0, 0, 0, 0, 0);
      } else if (g < n2) {
        // lane k == 0 of a link holds the link's parking queue
        const int gid = (int)(g - n1);
        const int4 info = S.lane_info[gid];
        if (lmeta_k((uint32_t)info.y) == 0)
          for (int q = S.lane_qhead[gid]; q < info.w; ++q) {
            const int id = S.wait_rec[q].x;
            h += veh_hash(id, kWaiting, 0, 0, 0, 0, 0) -
                 veh_hash(id, kArrived, 0, 0, 0, 0, 0);
            ++wait;
          }
      } else if (g < n3) {
        const int gid = (int)(g - n2);
        const int4 info = S.lane_info[gid];
        // the current state: buffer t & 1 of a fused slot; the handoffs of
        // the last step: buffer (t - 1) & 1
        const long long cur = S.fused ? (long long)(S.t & 1) * S.n_lanes : 0;
        const long long hpv =
            S.fused ? (long long)((S.t - 1) & 1) * S.n_lanes : 0;
        const int hc = S.lane_state[cur + gid].w;
        const int link = info.z;
        const int k = lmeta_k((uint32_t)info.y);
        const int len = lmeta_len((uint32_t)info.y);
        const int base = info.x;
        for (int j = 0; j < hc_cnt(hc); ++j) {
          const int slot = rec_slot(base, hc, len, j);
          const uint2 hw = S.hot[slot];
          const int id = (int)hw.y;
          const int rptr = (int)(S.cold[slot].x - S.route_off[id]);
          h += veh_hash(id, kActive, S.link_ext[link], k, xvf_x(hw.x),
                        xvf_v(hw.x), rptr) -
               veh_hash(id, kArrived, 0, 0, 0, 0, 0);
        }
        act += hc_cnt(hc);
        // a vehicle handed over in the last step is on this lane already
        const int4 ha = S.hand_a[hpv + gid];
        if (ha.x == S.t - 1) {
          const int id = ha.z;
          h += veh_hash(id, kActive, S.link_ext[link], k, xvf_x((uint32_t)ha.y),
                        xvf_v((uint32_t)ha.y), (int)(ha.w - S.route_off[id])) -
               veh_hash(id, kArrived, 0, 0, 0, 0, 0);
          ++act;
        }
      } else if (g < n4) {
        const long long tile = g - n3;
        for (int c = 0; c < C_N; ++c)
          atomicAdd(&out[c], (unsigned long long)S.tile_ctr[tile * C_N + c]);
      } else {
        const long long tile = g - n4;
        for (int c = 0; c < C_N; ++c)
          atomicAdd(&out[c], (unsigned long long)S.ftile_ctr[tile * C_N + c]);
      }
    }
  }
  atomicAdd(&out[C_N], act);
  atomicAdd(&out[C_N + 1], h);
  atomicAdd(&out[C_N + 2], wait);
}

__global__ void k_export_fill(ExportBufs o, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  o.status[i] = kArrived;
  o.link[i] = -1;
  o.lane[i] = 0;
  o.x[i] = 0;
  o.v[i] = 0;
  o.rptr[i] = 0;
}

__global__ void k_export_set(const DevScen* d, ExportBufs o, int ring) {
  const DevScen& S = *d;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (ring) {
    if (g >= S.ring_n) return;
    const int id = S.ring_id[g];
    o.status[id] = kActive;
    o.link[id] = 0;
    o.x[id] = S.ring_x[g];
    o.v[id] = (int8_t)S.ring_v[g];
    return;
  }
  if (g < S.n_lanes) {
    const int4 info = S.lane_info[g];
    if (lmeta_k((uint32_t)info.y) == 0)
      for (int q = S.lane_qhead[g]; q < info.w; ++q)
        o.status[S.wait_rec[q].x] = kWaiting;
  } else if (g < 2 * S.n_lanes) {
    const int gid = g - S.n_lanes;
    const long long cur = S.fused ? (long long)(S.t & 1) * S.n_lanes : 0;
    const long long hpv = S.fused ? (long long)((S.t - 1) & 1) * S.n_lanes : 0;
    const int hc = S.lane_state[cur + gid].w;
    const int4 info = S.lane_info[gid];
    const int link = info.z;
    const int k = lmeta_k((uint32_t)info.y);
    const int len = lmeta_len((uint32_t)info.y);
    const int base = info.x;
    for (int j = 0; j < hc_cnt(hc); ++j) {
      const int slot = rec_slot(base, hc, len, j);
      const uint2 hw = S.hot[slot];
      const int id = (int)hw.y;
      o.status[id] = kActive;
      o.link[id] = S.link_ext[link];
      o.lane[id] = (int8_t)k;
      o.x[id] = xvf_x(hw.x);
      o.v[id] = (int8_t)xvf_v(hw.x);
      o.rptr[id] = (int)(S.cold[slot].x - S.route_off[id]);
    }
    const int4 ha = S.hand_a[hpv + gid];
    if (ha.x == S.t - 1) {  // handed over in the last step
      const int id = ha.z;
      o.status[id] = kActive;
      o.link[id] = S.link_ext[link];
      o.lane[id] = (int8_t)k;
      o.x[id] = xvf_x((uint32_t)ha.y);
      o.v[id] = (int8_t)xvf_v((uint32_t)ha.y);
      o.rptr[id] = (int)(ha.w - S.route_off[id]);
    }
  }
}

// Each XCD's share of the lane-change kernel's work list, longest-running
// tile first.  The dispatcher deals list positions x, x + 8, x + 16, ... to
// XCD x, and a launch with more tiles than fit on the device at once ends
// late when a heavy tile starts late.  The heavy tiles of a congested
// network move with the congestion, so the order follows what each tile
// took in the front kernel since the list was last ordered (its cycle
// counter less the count snap holds for its position), not a fixed
// estimate.  Workgroup x sorts its positions in LDS (bitonic, descending;
// ties keep their order) and writes the items and their current counts
// back.  Which tile runs where changes no result.
__global__ __launch_bounds__(kOrderThreads) void k_order(
    const DevScen* __restrict__ descs, int4* __restrict__ work, int n,
    long long* __restrict__ snap) {
  __shared__ unsigned long long s_key[kOrderMax];
  __shared__ int4 s_item[kOrderMax];
  const int x = blockIdx.x;
  const int m = n > x ? (n - x + 7) / 8 : 0;  // this XCD's positions
  if (m > kOrderMax) return;  // (the host launches it only below that)
  auto cycles = [&](int4 w) {
    return descs[w.x].ftile_ctr[(long long)w.w * C_N + C_CYCLES];
  };
  for (int k = threadIdx.x; k < kOrderMax; k += kOrderThreads) {
    unsigned long long key = 0;  // padding sorts last
    if (k < m) {
      const int4 w = work[x + 8 * k];
      const long long d = cycles(w) - snap[x + 8 * k];
      const unsigned long long dt =
          d <= 0 ? 0ull : (d >= 0xFFFFFFFFll ? 0xFFFFFFFFull
                                            : (unsigned long long)d);
      key = (dt << 32) | (unsigned long long)(kOrderMax - k);
      s_item[k] = w;
    }
    s_key[k] = key;
  }
  for (int size = 2; size <= kOrderMax; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < kOrderMax / 2; t += kOrderThreads) {
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const unsigned long long a = s_key[lo], b = s_key[hi];
        if (desc ? a < b : a > b) {
          s_key[lo] = b;
          s_key[hi] = a;
        }
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += kOrderThreads) {
    const int k = kOrderMax - (int)(s_key[j] & 0xFFFFFFFFull);
    const int4 w = s_item[k];
    work[x + 8 * j] = w;
    snap[x + 8 * j] = cycles(w);
  }
}

// ---- launchers -------------------------------------------------------------

void* advance_kernel() { return reinterpret_cast<void*>(&k_advance); }
void* order_kernel() { return reinterpret_cast<void*>(&k_order); }

// Each launcher first clears any error left by earlier runtime calls of this
// thread, so that the status it returns is the launch's own.
hipError_t launch_advance(DevScen* d_descs, const int* d_slots, int n, int k,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_advance, dim3((n + 63) / 64), dim3(64), 0, s, d_descs,
                     d_slots, n, k);
  return hipGetLastError();
}

hipError_t launch_ring(DevScen* d_descs, const int* d_slots, int n,
                       int n_steps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_ring, dim3(n), dim3(kRingBlock), 0, s, d_descs,
                     d_slots, n_steps);
  return hipGetLastError();
}

hipError_t launch_stats(const DevScen* d_desc, unsigned long long* d_out,
                        int ring, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_stats, dim3(1024), dim3(256), 0, s, d_desc, d_out,
                     ring);
  return hipGetLastError();
}

hipError_t launch_export(const DevScen* d_desc, ExportBufs out, int n_veh,
                         int /*n_links*/, int n_lanes, int ring,
                         hipStream_t s) {
  (void)hipGetLastError();
  if (n_veh > 0)
    hipLaunchKernelGGL(k_export_fill, dim3((n_veh + 255) / 256), dim3(256), 0,
                       s, out, n_veh);
  const int n = ring ? n_veh : 2 * n_lanes;
  if (n > 0)
    hipLaunchKernelGGL(k_export_set, dim3((n + 255) / 256), dim3(256), 0, s,
                       d_desc, out, ring);
  return hipGetLastError();
}

}  // namespace tr
