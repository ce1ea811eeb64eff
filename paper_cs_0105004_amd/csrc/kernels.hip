// kernels.hip -- gfx950 kernels of the TRANSIMS per-second update.
//
// A step is two kernels, the GPU form of the paper's update sequence
// "change lanes / exchange / compute speeds and move / exchange" (Section
// "Micro-simulation parallelization: Domain decomposition"): the kernel
// boundaries are the two exchanges.  Each workgroup is one wavefront that
// owns a tile of whole links (at most 64 lanes); a lane's vehicles live in a
// lead-first ring buffer, so the per-step traffic is proportional to the
// vehicles, not to the cells.
//
//   k_front  (sub-step 1): merge the vehicle handed over by the upstream
//            node, let one vehicle per link leave parking, change lanes,
//            and publish per lane {target lane of the lead vehicle, x of the
//            rearmost vehicle}.
//   k_back   (sub-step 2): resolve each intersection from the published
//            summaries (priority by (rank, lane); the winner may drive
//            min(vmax, x_rear) cells into the next link), then accelerate,
//            brake to the gap, slow down at random and move every vehicle;
//            the lead vehicle that passes the node is written to the handoff
//            slot of its target lane (at most one per lane and step).
#include "kernels.h"
#include "philox.h"
#include "../../include/transims.h"

namespace tr {

namespace {

constexpr int kRingBlock = 256;

__device__ __forceinline__ int wrapi(int a, int cap) {
  return a >= cap ? a - cap : a;
}

// lane header word: head index (bits 0-15) and buffer parity (bit 16)
__device__ __forceinline__ int hp_head(int hp) { return hp & 0xFFFF; }
__device__ __forceinline__ int hp_par(int hp) { return hp >> 16; }

// record slot of the j-th vehicle (0 = lead) of a lane
__device__ __forceinline__ int rec_slot(int base, int hp, int len, int j) {
  return base + hp_par(hp) * len + wrapi(hp_head(hp) + j, len);
}

// flags of a vehicle entering `link` whose next route link is nxt (-1: none)
__device__ uint32_t route_flags(const DevScen& S, int link, int nxt) {
  int lo = 0, hi = S.link_lanes[link] - 1;
  if (nxt >= 0 && (S.flags & SIM_FLAG_TURN_LANES)) {
    for (int e = S.conn_off[link]; e < S.conn_off[link + 1]; ++e)
      if (S.conn_out[e] == nxt) {
        lo = S.conn_lo[e];
        hi = S.conn_hi[e];
        break;
      }
  }
  return fl_make(nxt < 0, lo, hi);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---- lane change on one tile ------------------------------------------
// Empty cells of lane m ahead of x up to the first vehicle or the link end,
// and behind x up to the first vehicle (cells before the link start count as
// empty), both capped at vmax.
__device__ __forceinline__ int lc_ahead(const short* lat, int len, int m,
                                        int x, int vmax) {
  int n = 0;
  for (int c = x + 1; c < len && n < vmax; ++c) {
    if (lat[m * len + c] >= 0) break;
    ++n;
  }
  return n;
}

__device__ __forceinline__ int lc_behind(const short* lat, int len, int m,
                                         int x, int vmax) {
  int n = 0;
  for (int c = x - 1; n < vmax; --c) {
    if (c >= 0 && lat[m * len + c] >= 0) break;
    ++n;
  }
  return n;
}

__device__ int lc_decide(const DevScen& S, const short* lat, int len,
                         int lanes, int k, int x, int v, uint32_t fl, int id,
                         int t) {
  const int vmax = S.vmax;
  const int lo = fl_lo(fl), hi = fl_hi(fl);
  if (k < lo || k > hi) {  // mandatory: one lane toward the turn lanes
    const int m = k < lo ? k + 1 : k - 1;
    const int need = min(vmax, (len - 1 - x) / S.lc_desp);
    if (lat[m * len + x] < 0 && lc_behind(lat, len, m, x, vmax) >= need)
      return m;
    return -1;
  }
  const int own = lc_ahead(lat, len, k, x, vmax);
  if (own >= min(v + 1, vmax)) return -1;
  int best = -1, best_a = -1;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int m = s == 0 ? k - 1 : k + 1;
    if (m < 0 || m >= lanes || m < lo || m > hi) continue;
    if (lat[m * len + x] >= 0) continue;
    const int a = lc_ahead(lat, len, m, x, vmax);
    if (a <= own) continue;
    if (lc_behind(lat, len, m, x, vmax) < vmax) continue;
    if (a > best_a) {
      best = m;
      best_a = a;
    }
  }
  if (best < 0) return -1;
  if ((uint64_t)veh_draw((uint32_t)id, (uint32_t)t, 0u, S.key0, S.key1) >=
      S.lc_thr)
    return -1;
  return best;
}

// Runs the lane-change sub-step on every multi-lane link of the tile.  The
// link's lanes are staged in LDS as a lattice of record offsets; movers are
// applied at once and, when any vehicle moved, the lanes' queues are
// rebuilt in the other half of their double buffer.
__device__ int lane_change_tile(const DevScen& S, int t, int2 tl, int* s_hp,
                                int* s_cnt, short* lat, signed char* dec) {
  const int i = threadIdx.x;
  int moves_total = 0;
  const int first_link = S.lane_link[tl.x];
  const int last_link = S.lane_link[tl.x + tl.y - 1];
  for (int link = first_link; link <= last_link; ++link) {
    const int lanes = S.link_lanes[link];
    if (lanes < 2) continue;
    const int lane0 = S.link_lane0[link];
    const int tb = lane0 - tl.x;
    int pre[5];
    pre[0] = 0;
    for (int k = 0; k < lanes; ++k) pre[k + 1] = pre[k] + s_cnt[tb + k];
    const int total = pre[lanes];
    if (total == 0) continue;
    const int len = S.link_len[link];
    const int region = S.lane_base[lane0];
    const int cells = lanes * len;
    for (int c = i; c < cells; c += kWave) {
      lat[c] = -1;
      dec[c] = -1;
    }
    __syncthreads();
    for (int f = i; f < total; f += kWave) {
      int k = 0;
      while (f >= pre[k + 1]) ++k;
      const int slot = rec_slot(S.lane_base[lane0 + k], s_hp[tb + k], len,
                                f - pre[k]);
      lat[k * len + xvf_x(S.hot[slot].x)] = (short)(slot - region);
    }
    __syncthreads();
    for (int f = i; f < total; f += kWave) {
      int k = 0;
      while (f >= pre[k + 1]) ++k;
      const int slot = rec_slot(S.lane_base[lane0 + k], s_hp[tb + k], len,
                                f - pre[k]);
      const uint2 hw = S.hot[slot];
      const int x = xvf_x(hw.x);
      const int d = lc_decide(S, lat, len, lanes, k, x, xvf_v(hw.x),
                              xvf_fl(hw.x), (int)hw.y, t);
      if (d >= 0) dec[k * len + x] = (signed char)d;
    }
    __syncthreads();
    // two movers into one cell come from both sides of it: the one from the
    // lower lane moves, the one moving left stays
    for (int c = i; c < cells; c += kWave) {
      const int d = dec[c];
      if (d < 0) continue;
      const int k = c / len, x = c - (c / len) * len;
      if (d == k - 1 && d - 1 >= 0 && dec[(d - 1) * len + x] == d)
        dec[c] = -2;
    }
    __syncthreads();
    int moved = 0;
    for (int c = i; c < cells; c += kWave) {
      const int d = dec[c];
      if (d < 0) continue;
      const int x = c - (c / len) * len;
      lat[d * len + x] = lat[c];
      lat[c] = -1;
      ++moved;
    }
    moved = (int)wave_sum((unsigned long long)moved);
    __syncthreads();
    if (moved > 0) {
      const int npar = 1 - hp_par(s_hp[tb]);
      for (int k = 0; k < lanes; ++k) {
        const int dst0 = S.lane_base[lane0 + k] + npar * len;
        int n = 0;
        for (int c0 = 0; c0 < len; c0 += kWave) {
          const int x = len - 1 - (c0 + i);
          const short o = x >= 0 ? lat[k * len + x] : (short)-1;
          const unsigned long long m = __ballot(o >= 0);
          if (o >= 0) {
            const int j = n + __popcll(m & ((1ull << i) - 1ull));
            S.hot[dst0 + j] = S.hot[region + o];
            S.cold[dst0 + j] = S.cold[region + o];
          }
          n += __popcll(m);
        }
        if (i == 0) {
          s_hp[tb + k] = npar << 16;
          s_cnt[tb + k] = n;
        }
      }
      __syncthreads();
      moves_total += moved;
    }
  }
  return moves_total;
}

}  // namespace

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kWave) void k_front(
    const DevScen* __restrict__ descs, const int2* __restrict__ work,
    int step) {
  extern __shared__ unsigned char dyn[];
  __shared__ int s_hp[kMaxTileLanes], s_cnt[kMaxTileLanes];
  const long long c0 = wall_clock64();
  const int2 w = work[blockIdx.x];
  const DevScen& S = descs[w.x];
  const int t = S.t + step;
  const int2 tl = S.tile_lanes[w.y];
  const int i = threadIdx.x;
  const bool act = i < tl.y;
  const int gid = tl.x + i;

  int hp = 0, cnt = 0, link = 0, k = 0, len = 1, base = 0, lanes = 1,
      lane0 = 0;
  uint32_t rear_w = 0;
  bool empty0 = false;
  if (act) {
    const int2 hc = S.lane_hc[gid];
    hp = hc.x;
    cnt = hc.y;
    link = S.lane_link[gid];
    lane0 = S.link_lane0[link];
    k = gid - lane0;
    len = S.link_len[link];
    base = S.lane_base[gid];
    lanes = S.link_lanes[link];
    // the vehicle the upstream node handed over in the previous step
    const int4 ha = S.hand_a[gid];
    if (ha.x == t - 1) {
      if (cnt >= len) {
        atomicOr(S.err, SIM_DEVERR_LANE_FULL);
      } else {
        const int slot = rec_slot(base, hp, len, cnt);
        S.hot[slot] = make_uint2((uint32_t)ha.y, (uint32_t)ha.z);
        S.cold[slot] = make_int2(ha.w, S.hand_nxt[gid]);
        ++cnt;
      }
    }
    empty0 = true;
    if (cnt > 0) {
      rear_w = S.hot[rec_slot(base, hp, len, cnt - 1)].x;
      empty0 = xvf_x(rear_w) != 0;
    }
  }
  // parking: the lowest lane of the link whose cell 0 is empty takes the
  // head of the link's queue if it has departed
  const unsigned long long free0 = __ballot(act && empty0);
  int ins = 0;
  if (act && empty0) {
    const unsigned long long lm =
        (free0 >> (lane0 - tl.x)) & ((1ull << lanes) - 1ull);
    if (__builtin_ctzll(lm) == k) {
      const int h = S.wait_head[link];
      if (h < S.wait_off[link + 1] && S.wait_dep[h] <= t) {
        const int id = S.wait_id[h];
        S.wait_head[link] = h + 1;
        const long long rp = S.route_off[id];
        const int nxt =
            rp + 1 < S.route_off[id + 1] ? S.route_links[rp + 1] : -1;
        rear_w = pack_xvf(0, 0, route_flags(S, link, nxt));
        const int slot = rec_slot(base, hp, len, cnt);
        S.hot[slot] = make_uint2(rear_w, (uint32_t)id);
        S.cold[slot] = make_int2((int)rp, nxt);
        ++cnt;
        ins = 1;
      }
    }
  }
  int lc_moves = 0;
  if (S.flags & SIM_FLAG_LANE_CHANGE) {
    if (act) {
      s_hp[i] = hp;
      s_cnt[i] = cnt;
    }
    __syncthreads();
    short* lat = reinterpret_cast<short*>(dyn);
    signed char* dec =
        reinterpret_cast<signed char*>(dyn) + (size_t)2 * S.lc_cells;
    lc_moves = lane_change_tile(S, t, tl, s_hp, s_cnt, lat, dec);
    __syncthreads();
    if (act) {
      hp = s_hp[i];
      cnt = s_cnt[i];
      if (cnt > 0) rear_w = S.hot[rec_slot(base, hp, len, cnt - 1)].x;
    }
  }
  if (act) {
    int tgt = -1, rear_x = len;
    if (cnt > 0) {
      rear_x = xvf_x(rear_w);
      const int ls = rec_slot(base, hp, len, 0);
      const uint32_t lw = S.hot[ls].x;
      if (len - 1 - xvf_x(lw) < S.vmax) {
        if (xvf_fl(lw) & kFlLast) {
          tgt = -2;
        } else {
          const int nxt = S.cold[ls].y;
          tgt = S.link_lane0[nxt] + min(k, (int)S.link_lanes[nxt] - 1);
        }
      }
    }
    S.lane_sum[gid] = make_int2(tgt, rear_x);
    S.lane_hc[gid] = make_int2(hp, cnt);
  }
  const unsigned long long n_ins = wave_sum((unsigned long long)ins);
  if (i == 0) {
    long long* ctr = S.tile_ctr + (long long)w.y * C_N;
    ctr[C_INS] += (long long)n_ins;
    ctr[C_LC] += lc_moves;
    ctr[C_CYCLES] += wall_clock64() - c0;
  }
}

__global__ __launch_bounds__(kWave) void k_back(
    const DevScen* __restrict__ descs, const int2* __restrict__ work,
    int step) {
  __shared__ int s_pre[kMaxTileLanes + 1];
  __shared__ int s_base[kMaxTileLanes], s_hp[kMaxTileLanes],
      s_len[kMaxTileLanes], s_extra[kMaxTileLanes], s_tgt[kMaxTileLanes],
      s_left[kMaxTileLanes];
  const long long c0 = wall_clock64();
  const int2 w = work[blockIdx.x];
  const DevScen& S = descs[w.x];
  const int t = S.t + step;
  const int vmax = S.vmax;
  const int2 tl = S.tile_lanes[w.y];
  const int nl = tl.y;
  const int i = threadIdx.x;
  const bool act = i < nl;
  const int gid = tl.x + i;

  int cnt = 0, len = 1, hp = 0;
  if (act) {
    const int2 hc = S.lane_hc[gid];
    hp = hc.x;
    cnt = hc.y;
    const int link = S.lane_link[gid];
    const int k = gid - S.link_lane0[link];
    len = S.link_len[link];
    const int2 sum = S.lane_sum[gid];
    int extra = 0;
    if (sum.x == -2) {
      extra = vmax;  // the trip ends at this node
    } else if (sum.x >= 0) {
      // priority: the candidate with the smallest (rank, lane) aiming at the
      // same target lane wins; in-links are sorted by rank
      const int node = S.link_to[link];
      const int mykey = S.link_rank[link] * 8 + k;
      bool win = true;
      for (int e = S.node_in_off[node]; e < S.node_in_off[node + 1] && win;
           ++e) {
        const int l2 = S.node_in[e];
        const int r2 = S.link_rank[l2] * 8;
        if (r2 > mykey) break;
        const int b2 = S.link_lane0[l2];
        const int n2 = S.link_lanes[l2];
        for (int k2 = 0; k2 < n2 && r2 + k2 < mykey; ++k2)
          if (S.lane_sum[b2 + k2].x == sum.x) {
            win = false;
            break;
          }
      }
      if (win) extra = min(vmax, S.lane_sum[sum.x].y);
    }
    s_base[i] = S.lane_base[gid];
    s_hp[i] = hp;
    s_len[i] = len;
    s_extra[i] = extra;
    s_tgt[i] = sum.x;
    s_left[i] = 0;
  }
  // exclusive prefix of the lane counts
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (i >= off) incl += y;
  }
  const int total = __shfl(incl, kWave - 1);
  if (act) s_pre[i] = incl - cnt;
  if (i == 0) s_pre[nl] = total;
  const unsigned long long cocc =
      wave_sum((unsigned long long)(cnt > 0 ? len : 0));
  __syncthreads();

  unsigned long long sumv = 0, cross = 0, exits = 0;
  // chunks from the rear so that every vehicle reads the position of the one
  // ahead before that one is rewritten
  for (int f0 = total > 0 ? ((total - 1) / kWave) * kWave : -1; f0 >= 0;
       f0 -= kWave) {
    const int f = f0 + i;
    if (f < total) {
      int lo = 0, hi = nl;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[mid] <= f) lo = mid;
        else hi = mid;
      }
      const int li = lo;
      const int j = f - s_pre[li];
      const int llen = s_len[li], lbase = s_base[li], lhp = s_hp[li];
      const int slot = rec_slot(lbase, lhp, llen, j);
      const uint2 hw = S.hot[slot];
      const int x = xvf_x(hw.x), v = xvf_v(hw.x);
      const uint32_t fl = xvf_fl(hw.x);
      int gap;
      if (j > 0) {
        gap = xvf_x(S.hot[rec_slot(lbase, lhp, llen, j - 1)].x) - x - 1;
      } else {
        gap = llen - 1 - x + s_extra[li];
      }
      const int v1 = min(v + 1, vmax);
      const int v2 = min(v1, gap);
      const uint32_t u = veh_draw(hw.y, (uint32_t)t, 1u, S.key0, S.key1);
      const int v3 = (v2 > 0 && (uint64_t)u < S.slow_thr) ? v2 - 1 : v2;
      const int nx = x + v3;
      sumv += v3;
      if (nx < llen) {
        S.hot[slot].x = pack_xvf(nx, v3, fl);
      } else {  // only the lead vehicle can pass the node
        const int2 cw = S.cold[slot];
        S.exit_t[cw.x] = t;
        s_left[li] = 1;
        if (fl & kFlLast) {
          ++exits;
        } else {
          const int id = (int)hw.y;
          const int nl2 = cw.y;
          const int nn = (long long)cw.x + 2 < S.route_off[id + 1]
                             ? S.route_links[cw.x + 2]
                             : -1;
          const int tgt = s_tgt[li];
          S.hand_nxt[tgt] = nn;
          S.hand_a[tgt] = make_int4(
              t, (int)pack_xvf(nx - llen, v3, route_flags(S, nl2, nn)), id,
              cw.x + 1);
          ++cross;
        }
      }
    }
  }
  __syncthreads();
  if (act && s_left[i]) {
    const int h = wrapi(hp_head(hp) + 1, len);
    S.lane_hc[gid] = make_int2((hp & ~0xFFFF) | h, cnt - 1);
  }
  sumv = wave_sum(sumv);
  cross = wave_sum(cross);
  exits = wave_sum(exits);
  if (i == 0) {
    long long* ctr = S.tile_ctr + (long long)w.y * C_N;
    ctr[C_UPDATES] += total;
    ctr[C_SUMV] += (long long)sumv;
    ctr[C_CROSS] += (long long)cross;
    ctr[C_EXITS] += (long long)exits;
    ctr[C_COCC] += (long long)cocc;
    ctr[C_CYCLES] += wall_clock64() - c0;
  }
}

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
    const long long n1 = S.n_veh, n2 = n1 + S.n_links, n3 = n2 + S.n_lanes,
                    n4 = n3 + S.n_tiles;
    for (long long g = g0; g < n4; g += stride) {
      if (g < n1) {
        h += veh_hash((int)g, kArrived, 0, 0, 0, 0, 0);
      } else if (g < n2) {
        const int link = (int)(g - n1);
        for (int q = S.wait_head[link]; q < S.wait_off[link + 1]; ++q) {
          const int id = S.wait_id[q];
          h += veh_hash(id, kWaiting, 0, 0, 0, 0, 0) -
               veh_hash(id, kArrived, 0, 0, 0, 0, 0);
          ++wait;
        }
      } else if (g < n3) {
        const int gid = (int)(g - n2);
        const int2 hc = S.lane_hc[gid];
        const int link = S.lane_link[gid];
        const int k = gid - S.link_lane0[link];
        const int len = S.link_len[link];
        const int base = S.lane_base[gid];
        for (int j = 0; j < hc.y; ++j) {
          const int slot = rec_slot(base, hc.x, len, j);
          const uint2 hw = S.hot[slot];
          const int id = (int)hw.y;
          const int rptr = (int)(S.cold[slot].x - S.route_off[id]);
          h += veh_hash(id, kActive, S.link_ext[link], k, xvf_x(hw.x),
                        xvf_v(hw.x), rptr) -
               veh_hash(id, kArrived, 0, 0, 0, 0, 0);
        }
        act += hc.y;
        // a vehicle handed over in the last step is on this lane already
        const int4 ha = S.hand_a[gid];
        if (ha.x == S.t - 1) {
          const int id = ha.z;
          h += veh_hash(id, kActive, S.link_ext[link], k, xvf_x((uint32_t)ha.y),
                        xvf_v((uint32_t)ha.y), (int)(ha.w - S.route_off[id])) -
               veh_hash(id, kArrived, 0, 0, 0, 0, 0);
          ++act;
        }
      } else {
        const long long tile = g - n3;
        for (int c = 0; c < C_N; ++c)
          atomicAdd(&out[c], (unsigned long long)S.tile_ctr[tile * C_N + c]);
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
  if (g < S.n_links) {
    for (int q = S.wait_head[g]; q < S.wait_off[g + 1]; ++q)
      o.status[S.wait_id[q]] = kWaiting;
  } else if (g < S.n_links + S.n_lanes) {
    const int gid = g - S.n_links;
    const int2 hc = S.lane_hc[gid];
    const int link = S.lane_link[gid];
    const int k = gid - S.link_lane0[link];
    const int len = S.link_len[link];
    const int base = S.lane_base[gid];
    for (int j = 0; j < hc.y; ++j) {
      const int slot = rec_slot(base, hc.x, len, j);
      const uint2 hw = S.hot[slot];
      const int id = (int)hw.y;
      o.status[id] = kActive;
      o.link[id] = S.link_ext[link];
      o.lane[id] = (int8_t)k;
      o.x[id] = xvf_x(hw.x);
      o.v[id] = (int8_t)xvf_v(hw.x);
      o.rptr[id] = (int)(S.cold[slot].x - S.route_off[id]);
    }
    const int4 ha = S.hand_a[gid];
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

// ---- launchers -------------------------------------------------------------

// Each launcher first clears any error left by earlier runtime calls of this
// thread, so that the status it returns is the launch's own.
hipError_t launch_front(const DevScen* d_descs, const int2* d_work, int n_work,
                        int step, int lc_cells, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_front, dim3(n_work), dim3(kWave), (size_t)3 * lc_cells,
                     s, d_descs, d_work, step);
  return hipGetLastError();
}

hipError_t launch_back(const DevScen* d_descs, const int2* d_work, int n_work,
                       int step, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_back, dim3(n_work), dim3(kWave), 0, s, d_descs, d_work,
                     step);
  return hipGetLastError();
}

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
                         int n_links, int n_lanes, int ring, hipStream_t s) {
  (void)hipGetLastError();
  if (n_veh > 0)
    hipLaunchKernelGGL(k_export_fill, dim3((n_veh + 255) / 256), dim3(256), 0,
                       s, out, n_veh);
  const int n = ring ? n_veh : n_links + n_lanes;
  if (n > 0)
    hipLaunchKernelGGL(k_export_set, dim3((n + 255) / 256), dim3(256), 0, s,
                       d_desc, out, ring);
  return hipGetLastError();
}

}  // namespace tr
