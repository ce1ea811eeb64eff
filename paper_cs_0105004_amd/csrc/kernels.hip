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
#include "transims.h"

namespace tr {

namespace {

constexpr int kRingBlock = 256;
// load of a lane in the move sub-step: its vehicles plus a fixed cost; a
// tile gets one move wavefront per kPieceCost of load (up to a limit)
constexpr int kLaneCost = 4;
constexpr int kPieceCost = 512;

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

// ---- lane change on one tile ------------------------------------------
// The lane-change sub-step of a tile works on bit lattices in LDS, one bit
// per cell.  Each lane of a link that changes lanes is padded to whole
// 32-bit words, so word q of lane k and word q of lane k +- 1 (q +- wpl)
// cover the same cells.  Per word of the tile (kLcBytesPerWord bytes):
//   occ  occupied cells before the sub-step; after the decisions, after it
//   rgt  vehicles moving one lane up (k -> k+1)
//   lft  vehicles moving one lane down (k -> k-1)
//   pre  running count of the new occupancy over the tile's words, mod 2^16
//        (a lane holds at most 32767 vehicles, so differences within one
//        lane are exact)
struct LcLat {
  uint32_t* occ;
  uint32_t* rgt;
  uint32_t* lft;
  uint16_t* pre;
};

// cells [c, c+32) of a lane of wpl words at w, cell c at bit 0; cells
// outside the lane read as empty (c may be negative)
__device__ __forceinline__ uint32_t lane_bits(const uint32_t* w, int wpl,
                                              int c) {
  const int q = c >> 5, sh = c & 31;
  const uint32_t lo = (q >= 0 && q < wpl) ? w[q] : 0u;
  const uint32_t hi = (q + 1 >= 0 && q + 1 < wpl) ? w[q + 1] : 0u;
  return sh == 0 ? lo : (lo >> sh) | (hi << (32 - sh));
}

__device__ __forceinline__ bool lane_bit(const uint32_t* w, int x) {
  return (w[x >> 5] >> (x & 31)) & 1u;
}

// Empty cells of a lane ahead of x up to the first vehicle or the link end,
// and behind x up to the first vehicle (cells before the link start count as
// empty), both capped at vmax (at most 7).
__device__ __forceinline__ int lc_ahead(const uint32_t* w, int wpl, int len,
                                        int x, int vmax) {
  const int lim = min(vmax, len - 1 - x);
  return (int)__builtin_ctz(lane_bits(w, wpl, x + 1) | (1u << lim));
}

__device__ __forceinline__ int lc_behind(const uint32_t* w, int wpl, int x,
                                         int vmax) {
  const uint32_t b = lane_bits(w, wpl, x - vmax) & ((1u << vmax) - 1u);
  return b == 0u ? vmax : vmax - 1 - (31 - (int)__builtin_clz(b));
}

// Target lane of the vehicle at cell x of lane k, or -1; wk: lane k's words
__device__ int lc_decide(const DevScen& S, const uint32_t* wk, int wpl,
                         int len, int lanes, int k, int x, int v, uint32_t fl,
                         int id, int t) {
  const int vmax = S.vmax;
  const int lo = fl_lo(fl), hi = fl_hi(fl);
  if (k < lo || k > hi) {  // mandatory: one lane toward the turn lanes
    const int m = k < lo ? k + 1 : k - 1;
    const uint32_t* wm = wk + (m - k) * wpl;
    const int need = min(vmax, (len - 1 - x) / S.lc_desp);
    if (!lane_bit(wm, x) && lc_behind(wm, wpl, x, vmax) >= need) return m;
    return -1;
  }
  const int own = lc_ahead(wk, wpl, len, x, vmax);
  if (own >= min(v + 1, vmax)) return -1;
  int best = -1, best_a = -1;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int m = s == 0 ? k - 1 : k + 1;
    if (m < 0 || m >= lanes || m < lo || m > hi) continue;
    const uint32_t* wm = wk + (m - k) * wpl;
    if (lane_bit(wm, x)) continue;
    const int a = lc_ahead(wm, wpl, len, x, vmax);
    if (a <= own) continue;
    if (lc_behind(wm, wpl, x, vmax) < vmax) continue;
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

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int i = threadIdx.x;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int u = __shfl_up(v, off);
    if (i >= off) v += u;
  }
  return v;
}

// Largest j < n with pre[j] <= f (pre ascending, pre[0] = 0 <= f)
__device__ __forceinline__ int lc_find(const int* pre, int n, int f) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= f) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Per-lane LDS of the tile for the lane-change sub-step
struct LcTile {
  const int4* info;  // lane_info of the tile's lanes
  int* hp;           // queue word (head, parity)
  int* cnt;          // vehicles
  int* wo;           // first lattice word (lanes that change lanes)
  int* vp;           // first vehicle in the tile's vehicle numbering
  int* mv;           // at a link's lane 0: 1 if any of its vehicles moved
  uint32_t* lw;      // lead record's xvf word after the sub-step
  int* lni;          // lead record's route word after the sub-step
  uint32_t* rw;      // rear record's xvf word after the sub-step
};

// Lane, record slot and xvf word of vehicle f of the tile's lattice
// (f < V; lanes in order, each lane lead first)
__device__ __forceinline__ void lc_locate(const LcTile& T, int nl, int f,
                                          int& ln, int& slot) {
  ln = lc_find(T.vp, nl, f);
  slot = rec_slot(T.info[ln].x, T.hp[ln], lmeta_len((uint32_t)T.info[ln].y),
                  f - T.vp[ln]);
}

// Vehicles per thread whose records stay in registers through the
// sub-step (the tile's first kLcRes * kWave vehicles: one round of loads);
// the rest are loaded again by each phase, kLcBatch per thread at a time.
constexpr int kLcRes = 2;
constexpr int kLcBatch = 2;

__device__ __forceinline__ void lc_mark_occ(const LcTile& T, const LcLat& Z,
                                            int ln, uint32_t xw) {
  const int x = xvf_x(xw);
  atomicOr(&Z.occ[T.wo[ln] + (x >> 5)], 1u << (x & 31));
}

__device__ __forceinline__ void lc_mark_move(const DevScen& S, const LcTile& T,
                                             const LcLat& Z, int t, int ln,
                                             v2u hw) {
  const uint32_t meta = (uint32_t)T.info[ln].y;
  const int len = lmeta_len(meta), k = lmeta_k(meta);
  const int wl = (len + 31) >> 5, q0 = T.wo[ln];
  const int x = xvf_x(hw.x);
  const int d = lc_decide(S, Z.occ + q0, wl, len, lmeta_lanes(meta), k, x,
                          xvf_v(hw.x), xvf_fl(hw.x), (int)hw.y, t);
  if (d < 0) return;
  atomicOr(d > k ? &Z.rgt[q0 + (x >> 5)] : &Z.lft[q0 + (x >> 5)],
           1u << (x & 31));
}

// Writes the vehicle's records at its place in its lane after the sub-step
// (links with a move only).
__device__ __forceinline__ void lc_place(const DevScen& S, const LcTile& T,
                                         const LcLat& Z, int ln, v2u hw,
                                         v2i cw) {
  const uint32_t meta = (uint32_t)T.info[ln].y;
  const int k = lmeta_k(meta);
  if (T.mv[ln - k] == 0) return;
  const int len = lmeta_len(meta), wl = (len + 31) >> 5;
  const int x = xvf_x(hw.x), b = x & 31;
  const int q = T.wo[ln] + (x >> 5);
  int d = 0;
  if ((Z.rgt[q] >> b) & 1u) d = 1;
  else if (((Z.lft[q] >> b) & 1u) &&
           !(k >= 2 && ((Z.rgt[q - 2 * wl] >> b) & 1u)))
    d = -1;
  const int lnd = ln + d, qd = q + d * wl;
  const int j = __popc(b == 31 ? 0u : Z.occ[qd] >> (b + 1)) +
                (int)(uint16_t)(Z.pre[T.wo[lnd] + wl - 1] - Z.pre[qd]);
  if (j >= len) {  // never: a lane holds at most len vehicles
    atomicOr(S.err, SIM_DEVERR_LANE_FULL);
    return;
  }
  const int npar = 1 - hc_par(T.hp[ln]);
  const int dst = T.info[lnd].x + npar * len + j;
  GAS v2u* hot = gpv<v2u>(S.hot);
  GAS v2i* cold = gpv<v2i>(S.cold);
  hot[dst] = hw;
  cold[dst] = cw;
  if (j == 0) {
    T.lw[lnd] = hw.x;
    T.lni[lnd] = cw.y;
  }
  if (j == T.cnt[lnd] - 1) T.rw[lnd] = hw.x;
}

// Runs the lane-change sub-step on every link of the tile that changes
// lanes (every decision on the lattice before the sub-step, then all moves
// at once).  A link any of whose vehicles moved has its lanes rebuilt, lead
// first, in the other half of their record double buffer; for those lanes
// T.hp, T.cnt, T.lw, T.lni and T.rw hold the new state.  Returns the number
// of vehicles that changed lanes.
__device__ int lane_change_tile(const DevScen& S, int t, int nl,
                                const LcTile& T, const LcLat& Z) {
  const int i = threadIdx.x;
  GAS v2u* hot = gpv<v2u>(S.hot);
  GAS v2i* cold = gpv<v2i>(S.cold);
  int wpl = 0, nv = 0, k = 0;
  if (i < nl) {
    const uint32_t meta = (uint32_t)T.info[i].y;
    if (lmeta_lanes(meta) >= 2) {
      wpl = (lmeta_len(meta) + 31) >> 5;
      nv = T.cnt[i];
      k = lmeta_k(meta);
    }
  }
  const int wi = wave_incl_scan(wpl), vi = wave_incl_scan(nv);
  const int Wt = __shfl(wi, kWave - 1), V = __shfl(vi, kWave - 1);
  if (V == 0) return 0;
  if (i < nl) {
    T.wo[i] = wi - wpl;
    T.vp[i] = vi - nv;
    T.mv[i] = 0;
  }
  for (int q = i; q < Wt; q += kWave) {
    Z.occ[q] = 0u;
    Z.rgt[q] = 0u;
    Z.lft[q] = 0u;
  }
  __syncthreads();

  // the first kLcRes * kWave vehicles, loaded once (threads past V load the
  // last vehicle and drop it)
  int rln[kLcRes];
  v2u rhw[kLcRes];
  v2i rcw[kLcRes];
  {
    int rsl[kLcRes];
#pragma unroll
    for (int u = 0; u < kLcRes; ++u)
      lc_locate(T, nl, min(u * kWave + i, V - 1), rln[u], rsl[u]);
#pragma unroll
    for (int u = 0; u < kLcRes; ++u) {
      rhw[u] = hot[rsl[u]];
      rcw[u] = cold[rsl[u]];
    }
  }
  const int f_rest = kLcRes * kWave;  // first vehicle of the loops below

  // occupancy
#pragma unroll
  for (int u = 0; u < kLcRes; ++u)
    if (u * kWave + i < V) lc_mark_occ(T, Z, rln[u], rhw[u].x);
  for (int f0 = f_rest; f0 < V; f0 += kLcBatch * kWave) {
    int ln[kLcBatch], sl[kLcBatch];
    uint32_t xw[kLcBatch];
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      lc_locate(T, nl, min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u) xw[u] = hot[sl[u]].x;
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      if (f0 + u * kWave + i < V) lc_mark_occ(T, Z, ln[u], xw[u]);
  }
  __syncthreads();

  // decisions
#pragma unroll
  for (int u = 0; u < kLcRes; ++u)
    if (u * kWave + i < V) lc_mark_move(S, T, Z, t, rln[u], rhw[u]);
  for (int f0 = f_rest; f0 < V; f0 += kLcBatch * kWave) {
    int ln[kLcBatch], sl[kLcBatch];
    v2u hw[kLcBatch];
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      lc_locate(T, nl, min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u) hw[u] = hot[sl[u]];
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      if (f0 + u * kWave + i < V) lc_mark_move(S, T, Z, t, ln[u], hw[u]);
  }
  __syncthreads();

  // two movers into one cell come from both sides of it: the one from the
  // lower lane moves, the one moving down stays.  occ becomes the occupancy
  // after the sub-step.
  int moved = 0;
  for (int q = i; q < Wt; q += kWave) {
    const int ln = lc_find(T.wo, nl, q);
    const uint32_t meta = (uint32_t)T.info[ln].y;
    const int kk = lmeta_k(meta), L = lmeta_lanes(meta);
    const int wl = (lmeta_len(meta) + 31) >> 5;
    const uint32_t up = Z.rgt[q];
    const uint32_t below = kk >= 1 ? Z.rgt[q - wl] : 0u;  // k-1 -> k
    const uint32_t down = Z.lft[q] & ~(kk >= 2 ? Z.rgt[q - 2 * wl] : 0u);
    const uint32_t above = kk + 1 < L ? Z.lft[q + wl] & ~below : 0u;
    Z.occ[q] = (Z.occ[q] & ~up & ~down) | below | above;
    const int m = __popc(up) + __popc(down);
    if (m) T.mv[ln - kk] = 1;
    moved += m;
  }
  moved = (int)wave_sum((unsigned long long)moved);
  if (moved == 0) return 0;
  int carry = 0;
  for (int q0 = 0; q0 < Wt; q0 += kWave) {
    const int q = q0 + i;
    const int c = wave_incl_scan(q < Wt ? __popc(Z.occ[q]) : 0);
    if (q < Wt) Z.pre[q] = (uint16_t)(carry + c);
    carry += __shfl(c, kWave - 1);
  }
  __syncthreads();
  const bool mine = wpl > 0 && T.mv[i - k] != 0;
  if (mine) {
    const int q0 = T.wo[i];
    T.cnt[i] = (int)(uint16_t)(Z.pre[q0 + wpl - 1] -
                               (q0 > 0 ? Z.pre[q0 - 1] : (uint16_t)0));
  }
  __syncthreads();

  // rebuild the lanes of the links that moved, lead first
#pragma unroll
  for (int u = 0; u < kLcRes; ++u)
    if (u * kWave + i < V) lc_place(S, T, Z, rln[u], rhw[u], rcw[u]);
  for (int f0 = f_rest; f0 < V; f0 += kLcBatch * kWave) {
    int ln[kLcBatch], sl[kLcBatch];
    v2u hw[kLcBatch];
    v2i cw[kLcBatch];
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      lc_locate(T, nl, min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u) {
      hw[u] = hot[sl[u]];
      cw[u] = cold[sl[u]];
    }
#pragma unroll
    for (int u = 0; u < kLcBatch; ++u)
      if (f0 + u * kWave + i < V) lc_place(S, T, Z, ln[u], hw[u], cw[u]);
  }
  __syncthreads();
  if (mine) T.hp[i] = hc_make(0, 1 - hc_par(T.hp[i]), 0);
  return moved;
}

}  // namespace

// ---------------------------------------------------------------------------
// Work items are {slot, first lane, lanes, tile}.  With kBatched false every
// item belongs to slot `slot`, whose descriptor is then read without waiting
// for the work item.

template <bool kBatched>
__global__ __launch_bounds__(kWave) void k_front(
    const DevScen* __restrict__ descs, int slot, const int4* __restrict__ work,
    int pieces, int step) {
  extern __shared__ unsigned char dyn[];
  __shared__ int4 s_info[kMaxTileLanes];
  __shared__ int s_hp[kMaxTileLanes], s_cnt[kMaxTileLanes];
  __shared__ int s_wo[kMaxTileLanes], s_vp[kMaxTileLanes], s_mv[kMaxTileLanes];
  __shared__ int s_lni[kMaxTileLanes];
  __shared__ uint32_t s_lw[kMaxTileLanes], s_rw[kMaxTileLanes];
  __shared__ int4 s_plans[kMaxPlans];
  const long long c0 = wall_clock64();
  const int4 w = work[blockIdx.x];
  const DevScen& S = descs[kBatched ? w.x : slot];
  const int t = S.t + step;
  const int vmax = S.vmax;
  const GAS v4i* __restrict__ lane_info = gpv<v4i>(S.lane_info);
  const GAS v4i* __restrict__ lane_state = gpv<v4i>(S.lane_state);
  GAS v4i* __restrict__ lane_sum = gpv<v4i>(S.lane_sum);
  GAS int32_t* __restrict__ claim_a = gp(S.claim);
  const GAS v4i* __restrict__ hand_a = gpv<v4i>(S.hand_a);
  const GAS int32_t* __restrict__ hand_b = gp(S.hand_b);
  GAS int32_t* __restrict__ lane_qhead = gp(S.lane_qhead);
  GAS v4i* __restrict__ lane_qrec = gpv<v4i>(S.lane_qrec);
  // the lane-change pass reaches the records through the descriptor too
  GAS v2u* hot = gpv<v2u>(S.hot);
  GAS v2i* cold = gpv<v2i>(S.cold);
  const int i = threadIdx.x;
  const int nl = w.z;
  const bool act = i < nl;
  const int gid = w.y + i;

  // everything this kernel reads of a lane, in one round of loads
  // (threads past the tile's lanes read its first lane and drop it, so
  // that no load waits behind a branch)
  const int gg = act ? gid : w.y;
  v4i info = lane_info[gg], st = lane_state[gg], ha = hand_a[gg];
  v4i qrec = lane_qrec[gg];
  int hb = hand_b[gg], qhead = lane_qhead[gg];
  if (!act) {
    info = (v4i){0, 0, 0, 0};
    st = (v4i){0, 0, 0, 0};
    ha = (v4i){0, 0, 0, 0};
    qrec = (v4i){-1, 0, 0, 0};
    hb = 0;
    qhead = 0;
  }
  load_plans(S, s_plans);
  const uint32_t meta = (uint32_t)info.y;
  const int len = act ? lmeta_len(meta) : 1;
  const int k = lmeta_k(meta), lanes = lmeta_lanes(meta);
  const int base = info.x;
  int head = hc_head(st.w), par = hc_par(st.w), cnt = act ? hc_cnt(st.w) : 0;
  uint32_t lead_w = (uint32_t)st.x, rear_w = (uint32_t)st.z;
  int lead_ninfo = st.y;

  // the vehicle the upstream node handed over in the previous step
  if (act && ha.x == t - 1) {
    if (cnt >= len) {
      atomicOr(S.err, SIM_DEVERR_LANE_FULL);
    } else {
      const int slot = rec_slot(base, st.w, len, cnt);
      hot[slot] = (v2u){(uint32_t)ha.y, (uint32_t)ha.z};
      cold[slot] = (v2i){ha.w, hb};
      rear_w = (uint32_t)ha.y;
      if (cnt == 0) {
        lead_w = rear_w;
        lead_ninfo = hb;
      }
      ++cnt;
    }
  }
  // parking: the lowest lane of the link whose cell 0 is empty takes the
  // head of the link's queue if it has departed.  The queue is kept with the
  // link's lane 0, whose thread shares it.
  const bool empty0 = act && (cnt == 0 || xvf_x(rear_w) != 0);
  const unsigned long long free0 = __ballot(empty0);
  const int l0 = i - k;  // this link's lane 0 in the tile
  const int qh = __shfl(qhead, l0);
  const int qid = __shfl(qrec.x, l0), qdep = __shfl(qrec.y, l0),
            qrp = __shfl(qrec.z, l0), qni = __shfl(qrec.w, l0);
  int ins = 0;
  if (empty0) {
    const unsigned long long lm = (free0 >> l0) & ((1ull << lanes) - 1ull);
    if (__builtin_ctzll(lm) == k && qh < info.w && qid >= 0 &&
        (qdep & ((1 << kDepartBits) - 1)) <= t) {
      rear_w = pack_xvf(0, 0, (uint32_t)qdep >> kDepartBits);
      const int slot = rec_slot(base, st.w, len, cnt);
      hot[slot] = (v2u){rear_w, (uint32_t)qid};
      cold[slot] = (v2i){qrp, qni};
      if (cnt == 0) {
        lead_w = rear_w;
        lead_ninfo = qni;
      }
      ++cnt;
      ins = 1;
    }
  }
  const unsigned long long insm = __ballot(ins);
  if (act && k == 0 && ((insm >> i) & ((1ull << lanes) - 1ull)) != 0) {
    lane_qhead[gid] = qhead + 1;
    lane_qrec[gid] = (v4i){-1, 0, 0, 0};  // the move kernel fetches the next
  }
  int lc_moves = 0;
  if (S.flags & SIM_FLAG_LANE_CHANGE) {
    if (act) {
      s_info[i] = make_int4(info.x, info.y, info.z, info.w);
      s_hp[i] = hc_make(head, par, 0);
      s_cnt[i] = cnt;
    }
    __syncthreads();
    const LcTile T{s_info, s_hp, s_cnt, s_wo, s_vp, s_mv, s_lw, s_lni, s_rw};
    uint32_t* occ = reinterpret_cast<uint32_t*>(dyn);
    const LcLat Z{occ, occ + S.lc_words, occ + 2 * S.lc_words,
                  reinterpret_cast<uint16_t*>(occ + 3 * S.lc_words)};
    lc_moves = lane_change_tile(S, t, nl, T, Z);
    __syncthreads();
    if (act && lc_moves > 0 && hc_make(head, par, 0) != s_hp[i]) {
      head = hc_head(s_hp[i]);
      par = hc_par(s_hp[i]);
      cnt = s_cnt[i];
      if (cnt > 0) {
        lead_w = s_lw[i];
        lead_ninfo = s_lni[i];
        rear_w = s_rw[i];
      }
    }
  }
  __syncthreads();  // the plans in LDS (and the lane-change pass's writes)
  if (act) {
    int tgt = -1;
    const int rear_x = cnt > 0 ? xvf_x(rear_w) : len;
    // a red light holds the lead vehicle back: no claim, no trip end
    if (cnt > 0 && len - 1 - xvf_x(lead_w) < vmax &&
        !sig_red(s_plans, meta, t)) {
      if (xvf_fl(lead_w) & kFlLast) {
        tgt = -2;  // the trip ends at this node
      } else {
        const uint32_t ni = (uint32_t)lead_ninfo;
        tgt = rinfo_lane0(ni) + min(k, rinfo_lanes(ni) - 1);
        // priority among the candidates aiming at one lane: smallest
        // (rank of the link, lane); they all enter the same node
        atomicMin((int*)&claim_a[tgt], lmeta_rank(meta) * 8 + k);
      }
    }
    lane_sum[gid] = (v4i){tgt, rear_x, hc_make(head, par, cnt), 0};
  }
  // runs of this tile for the move sub-step: a tile heavier than
  // kPieceCost gets more wavefronts, listed for the move kernel
  if (pieces > 1 && S.xcap > 0) {
    const unsigned long long T =
        wave_sum((unsigned long long)(act ? cnt + kLaneCost : 0));
    const int np = min(pieces, (int)((T + kPieceCost - 1) / kPieceCost));
    if (i == 0) {
      int got = 0;
      if (np > 1) {
        const int xb = atomicAdd(&S.xcount[t & 1], np - 1);
        got = max(0, min(S.xcap - xb, np - 1));
        for (int r = 0; r < got; ++r)
          S.xlist[xb + r] =
              make_int4(w.y, w.z | ((r + 1) << 8) | ((got + 1) << 16), w.w, 0);
      }
      S.tile_np[w.w] = got + 1;
    }
  }
  const unsigned long long n_ins = wave_sum((unsigned long long)ins);
  if (i == 0) {
    long long* ctr = S.ftile_ctr + (long long)w.w * C_N;
    if (n_ins) atomicAdd((unsigned long long*)&ctr[C_INS], n_ins);
    if (lc_moves) atomicAdd((unsigned long long*)&ctr[C_LC],
                            (unsigned long long)lc_moves);
    atomicAdd((unsigned long long*)&ctr[C_CYCLES],
              (unsigned long long)(wall_clock64() - c0));
  }
}

// Orders this lane's LDS accesses before the next ones of any lane of the
// wavefront: a wavefront executes its LDS instructions in order, so keeping
// the compiler from moving them is enough, and nothing waits on memory.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The back kernel: one wavefront per tile of at most 64 lanes, plus the
// extra wavefronts the front kernel listed for heavy tiles.  The wavefronts
// of a tile cut it into as many contiguous runs of lanes of about equal load
// (vehicles + kLaneCost per lane) -- the paper's load balancing by measured
// load, redone every step from the current counts -- and each takes one run.
// Lane threads resolve the intersections, then the vehicles of the run are
// updated 64 at a time.
constexpr int kGroup = 2;  // chunks of 64 vehicles loaded before updating

template <bool kBatched>
__global__ __launch_bounds__(kWave) void k_back(
    const DevScen* __restrict__ descs, int slot, const int4* __restrict__ work,
    int n_work, int step) {
  __shared__ int s_pre[kMaxTileLanes + 1];
  __shared__ int s_base[kMaxTileLanes], s_hp[kMaxTileLanes],
      s_len[kMaxTileLanes], s_key[kMaxTileLanes], s_tgt[kMaxTileLanes],
      s_left[kMaxTileLanes];
  __shared__ int4 s_ends[kMaxTileLanes];    // new lead xvf/ninfo, rear xvf
  __shared__ int2 s_second[kMaxTileLanes];  // the vehicle behind the lead
  const long long c0 = wall_clock64();
  // the next step's list of extra wavefronts starts empty (done before any
  // wavefront can leave early)
  if (!kBatched && blockIdx.x == 0 && threadIdx.x == 0 && descs[slot].xcap > 0)
    descs[slot].xcount[(descs[slot].t + step + 1) & 1] = 0;
  int4 w;
  int piece = 0, np = 1;
  if ((int)blockIdx.x < n_work) {
    w = work[blockIdx.x];
    if (!kBatched && descs[slot].xcap > 0) np = descs[slot].tile_np[w.w];
  } else {  // an extra wavefront of a heavy tile (single slot only)
    const DevScen& S1 = descs[slot];
    const int e = (int)blockIdx.x - n_work;
    const int t1 = S1.t + step;
    if (e >= min(S1.xcount[t1 & 1], S1.xcap)) return;
    const int4 x = S1.xlist[e];
    w = make_int4(slot, x.x, x.y & 0xFF, x.z);
    piece = (x.y >> 8) & 0xFF;
    np = x.y >> 16;
  }
  const DevScen& S = descs[kBatched ? w.x : slot];
  // everything the kernel touches, in registers, as global pointers
  const int t = S.t + step;
  const int vmax = S.vmax;
  const uint32_t key0 = S.key0, key1 = S.key1;
  const uint64_t slow_thr = S.slow_thr;
  const GAS v4i* __restrict__ lane_info = gpv<v4i>(S.lane_info);
  const GAS v4i* __restrict__ lane_sum = gpv<v4i>(S.lane_sum);
  GAS v4i* __restrict__ lane_state = gpv<v4i>(S.lane_state);
  GAS int32_t* __restrict__ lane_qhead = gp(S.lane_qhead);
  GAS v4i* __restrict__ lane_qrec = gpv<v4i>(S.lane_qrec);
  const GAS v4i* __restrict__ wait_rec = gpv<v4i>(S.wait_rec);
  GAS int32_t* __restrict__ claim_a = gp(S.claim);
  GAS v4i* __restrict__ hand_a = gpv<v4i>(S.hand_a);
  GAS int32_t* __restrict__ hand_b = gp(S.hand_b);
  // hot and hot_w name the same records (loads / xvf stores): no restrict
  GAS v2u* hot = gpv<v2u>(S.hot);
  GAS uint32_t* hot_w = gpv<uint32_t>(S.hot);  // word 0 of a record = xvf
  const GAS v2i* __restrict__ cold = gpv<v2i>(S.cold);
  const GAS uint32_t* __restrict__ route_info = gp(S.route_info);
  GAS int32_t* __restrict__ exit_t = gp(S.exit_t);
  // counters of a run live at the entry of its first lane (set below)
  GAS unsigned long long* __restrict__ ctr = nullptr;
  const int nl = w.z;
  const int i = threadIdx.x;
  const int gid = w.y + i;

  // The lane counts come from the summary the front kernel published: the
  // other wavefronts of this tile rewrite lane_hc of their own lanes while
  // this one may still be reading, so the split must not depend on it.
  int cnt = 0;
  v4i sum = {-1, 0, 0, 0};
  v4i info = {0, 0, 0, 0}, qrec = {0, 0, 0, 0};
  int qhead = 0;
  if (i < nl) {
    sum = lane_sum[gid];
    info = lane_info[gid];
    qhead = lane_qhead[gid];
    qrec = lane_qrec[gid];
  }
  // this wavefront's run of lanes
  bool act = false;
  {
    const int cost = i < nl ? hc_cnt(sum.z) + kLaneCost : 0;
    int ci = cost;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int y = __shfl_up(ci, off);
      if (i >= off) ci += y;
    }
    const int T = __builtin_amdgcn_readfirstlane(__shfl(ci, kWave - 1));
    const int id = (int)(((long long)(ci - cost) * np) / T);
    act = i < nl && id == piece;
    if (__ballot(act) == 0ull) return;  // no run for this wavefront
  }
  int len = 1, hp = 0;
  // a link's parking queue moved on in the front pass: fetch its new head
  // record now, store it at the end
  const bool refill = act && lmeta_k((uint32_t)info.y) == 0 && qrec.x < 0 &&
                      qhead < info.w;
  v4i nrec = {-1, 0, 0, 0};
  if (refill) nrec = wait_rec[qhead];
  if (act) {
    hp = sum.z;
    cnt = hc_cnt(sum.z);
    const uint32_t meta = (uint32_t)info.y;
    len = lmeta_len(meta);
    s_base[i] = info.x;
    s_hp[i] = hp;
    s_len[i] = len;
    s_tgt[i] = sum.x;
    s_key[i] = lmeta_rank(meta) * 8 + lmeta_k(meta);
    s_left[i] = 0;
    s_ends[i] = make_int4(0, 0, 0, 0);
  }
  // exclusive prefix of the run's lane counts (zero outside the run)
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (i >= off) incl += y;
  }
  // uniform across the wavefront: keep it in a scalar register
  const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1));
  // every lane of the tile gets its entry (lanes outside the run hold no
  // vehicles of it), so the search below only ever lands on the run's lanes
  if (i < nl) s_pre[i] = incl - cnt;
  if (i == 0) s_pre[nl] = total;
  const unsigned long long cocc =
      wave_sum((unsigned long long)(cnt > 0 ? len : 0));
  wave_lds_sync();

  unsigned long long sumv = 0, cross = 0, exits = 0;
  const int nchunk = (total + kWave - 1) / kWave;
  // Groups of chunks run from the rear: a group loads every record it needs
  // before rewriting any, so each vehicle reads the position of the one
  // ahead before it changes.
  for (int g0 = ((nchunk - 1) / kGroup) * kGroup; nchunk > 0 && g0 >= 0;
       g0 -= kGroup) {
    v2u hw[kGroup];
    v2i cw[kGroup];
    uint32_t ahead[kGroup];
    int sl[kGroup], lij[kGroup], clm[kGroup], rear[kGroup];
    {
      // Every thread loads (threads past the last vehicle repeat it), so no
      // load sits in a divergent branch and all of them stay in flight.
#pragma unroll
      for (int c = 0; c < kGroup; ++c) {
        const int fr = (g0 + c) * kWave + i;
        const int f = min(fr, total - 1);
        int lo = 0, hi = nl;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_pre[mid] <= f) lo = mid;
          else hi = mid;
        }
        const int j = f - s_pre[lo];
        const int llen = s_len[lo], lbase = s_base[lo], lhp = s_hp[lo];
        sl[c] = rec_slot(lbase, lhp, llen, j);
        // vehicles that need no neighbour / route state read their own
        // record or their lane's lead instead
        const int sa = j > 0 ? rec_slot(lbase, lhp, llen, j - 1) : sl[c];
        const int sc = j <= 1 ? sl[c] : rec_slot(lbase, lhp, llen, 0);
        // the lead of a lane near its node also fetches the claim on its
        // target lane and that lane's rearmost position
        const int tg = s_tgt[lo];
        const int q = (j == 0 && tg >= 0) ? tg : w.y + lo;
        hw[c] = hot[sl[c]];
        ahead[c] = hot_w[2 * sa];
        cw[c] = cold[sc];
        clm[c] = claim_a[q];
        rear[c] = lane_sum[q].y;
        lij[c] = fr < total ? (lo | (j << 8)) : -1;
      }
    }
#pragma unroll
    for (int c = 0; c < kGroup; ++c) {
      if (lij[c] < 0) continue;
      const int li = lij[c] & 0xFF, j = lij[c] >> 8;
      const int llen = s_len[li];
      const int x = xvf_x(hw[c].x), v = xvf_v(hw[c].x);
      const uint32_t fl = xvf_fl(hw[c].x);
      int extra = 0;  // cells the lead may drive past the link end
      if (j == 0) {
        const int tg = s_tgt[li];
        if (tg == -2) {
          extra = vmax;  // the trip ends at this node
        } else if (tg >= 0 && clm[c] == s_key[li]) {
          extra = min(vmax, rear[c]);  // priority among the candidates
          claim_a[tg] = INT32_MAX;     // the winner clears the claim
        }
      }
      const int gap = j > 0 ? xvf_x(ahead[c]) - x - 1 : llen - 1 - x + extra;
      const int v1 = min(v + 1, vmax);
      const int v2 = min(v1, gap);
      const uint32_t u = veh_draw(hw[c].y, (uint32_t)t, 1u, key0, key1);
      const int v3 = (v2 > 0 && (uint64_t)u < slow_thr) ? v2 - 1 : v2;
      const int nx = x + v3;
      sumv += v3;
      if (nx < llen) {
        const uint32_t nw = pack_xvf(nx, v3, fl);
        hot_w[2 * sl[c]] = nw;
        const int lcnt = s_pre[li + 1] - s_pre[li];
        if (j == 0) {
          s_ends[li].x = (int)nw;
          s_ends[li].y = cw[c].y;
        } else if (j == 1) {
          s_second[li] = make_int2((int)nw, cw[c].y);
        }
        if (j == lcnt - 1) s_ends[li].z = (int)nw;
      } else {  // only the lead vehicle can pass the node
        const int rp = cw[c].x;
        exit_t[rp] = t;
        s_left[li] = 1;
        if (fl & kFlLast) {
          ++exits;
        } else {
          const uint32_t nfl = rinfo_flags((uint32_t)cw[c].y);
          const int tg = s_tgt[li];
          hand_b[tg] = (nfl & kFlLast) ? 0 : (int)route_info[rp + 2];
          hand_a[tg] = (v4i){t, (int)pack_xvf(nx - llen, v3, nfl),
                             (int)hw[c].y, rp + 1};
          ++cross;
        }
      }
    }
  }
  wave_lds_sync();
  if (act) {
    int4 e = s_ends[i];
    int hc = hc_make(hc_head(hp), hc_par(hp), cnt);
    if (s_left[i]) {
      hc = hc_make(wrapi(hc_head(hp) + 1, len), hc_par(hp), cnt - 1);
      const int2 sec = s_second[i];
      e.x = sec.x;  // the vehicle behind is the new lead
      e.y = sec.y;
    }
    lane_state[gid] = (v4i){e.x, e.y, e.z, hc};
  }
  if (refill) lane_qrec[gid] = nrec;
  sumv = wave_sum(sumv);
  cross = wave_sum(cross);
  exits = wave_sum(exits);
  const int first = __builtin_amdgcn_readfirstlane(
      __builtin_ctzll(__ballot(act)));  // the run's first lane in the tile
  ctr = (GAS unsigned long long*)gp(S.tile_ctr + (long long)(w.y + first) * C_N);
  if (i == 0) {
    atomicAdd((unsigned long long*)&ctr[C_UPDATES], (unsigned long long)total);
    atomicAdd((unsigned long long*)&ctr[C_SUMV], sumv);
    if (cross) atomicAdd((unsigned long long*)&ctr[C_CROSS], cross);
    if (exits) atomicAdd((unsigned long long*)&ctr[C_EXITS], exits);
    atomicAdd((unsigned long long*)&ctr[C_COCC], cocc);
    atomicAdd((unsigned long long*)&ctr[C_CYCLES],
              (unsigned long long)(wall_clock64() - c0));
  }
}

// ---------------------------------------------------------------------------
// The move of one group of kGroup x 64 vehicles in the one-kernel step:
// step_load reads what the group needs (vehicle records from the lanes'
// rings, or from LDS for the vehicles that arrived in this step),
// step_run updates the group.
struct StepGroup {
  v2u hw[kGroup];
  v2i cw[kGroup];
  uint32_t ahead[kGroup];
  int sl[kGroup], lij[kGroup];
};
struct StepCtx {
  int t, vmax;
  uint32_t key0, key1;
  uint64_t slow_thr;
};

__device__ __forceinline__ void step_load(
    StepGroup& G, int g0, int i, int total, int nl, const int* s_pre,
    const int* s_len, const int* s_base, const int* s_hp, GAS v2u* hot,
    GAS uint32_t* hot_w, GAS v2i* cold) {
#pragma unroll
  for (int c = 0; c < kGroup; ++c) {
    const int fr = (g0 + c) * kWave + i;
    const int f = max(min(fr, total - 1), 0);
    int lo = 0, hi = nl;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pre[mid] <= f) lo = mid;
      else hi = mid;
    }
    const int j = f - s_pre[lo];
    const int llen = s_len[lo], lbase = s_base[lo], lhp = s_hp[lo];
    G.sl[c] = rec_slot(lbase, lhp, llen, j);
    // ring slots are loaded for every vehicle (an arrival's slot holds a
    // stale record, which step_run replaces from LDS), so no load sits in
    // a branch
    const int sa = j > 0 ? rec_slot(lbase, lhp, llen, j - 1) : G.sl[c];
    const int sc = j <= 1 ? G.sl[c] : rec_slot(lbase, lhp, llen, 0);
    G.hw[c] = hot[G.sl[c]];
    G.ahead[c] = hot_w[2 * sa];
    G.cw[c] = cold[sc];
    G.lij[c] = (fr < total) ? (lo | (j << 8)) : -1;
  }
}

__device__ __forceinline__ void step_run(
    const StepGroup& G, const StepCtx& cx, const int* s_len, const int* s_cnt0,
    const int* s_pre, const int* s_extra, const int* s_tgt,
    const uint2 (*s_nhot)[2], const int2 (*s_ncold)[2], int4* s_ends,
    int2* s_second, int* s_left, GAS v2u* hot, GAS uint32_t* hot_w,
    GAS v2i* cold, const GAS uint32_t* __restrict__ route_info,
    GAS int32_t* __restrict__ exit_t, GAS v4i* __restrict__ ha_out,
    GAS int32_t* __restrict__ hb_out, GAS int32_t* __restrict__ ht_out,
    unsigned long long& sumv, unsigned long long& cross,
    unsigned long long& exits) {
#pragma unroll
  for (int c = 0; c < kGroup; ++c) {
    if (G.lij[c] < 0) continue;
    const int li = G.lij[c] & 0xFF, j = G.lij[c] >> 8;
    const int llen = s_len[li];
    const int c0l = s_cnt0[li];
    v2u hw = G.hw[c];
    v2i cw = G.cw[c];
    uint32_t ahead = G.ahead[c];
    if (j >= c0l) {  // an arrival of this step
      const uint2 h = s_nhot[li][j - c0l];
      const int2 cc = s_ncold[li][j - c0l];
      hw = (v2u){h.x, h.y};
      cw = (v2i){cc.x, cc.y};
    }
    if (j > 0 && j - 1 >= c0l) ahead = s_nhot[li][j - 1 - c0l].x;
    const int x = xvf_x(hw.x), v = xvf_v(hw.x);
    const uint32_t fl = xvf_fl(hw.x);
    const int gap = j > 0 ? xvf_x(ahead) - x - 1 : llen - 1 - x + s_extra[li];
    const int v1 = min(v + 1, cx.vmax);
    const int v2 = min(v1, gap);
    const uint32_t u = veh_draw(hw.y, (uint32_t)cx.t, 1u, cx.key0, cx.key1);
    const int v3 = (v2 > 0 && (uint64_t)u < cx.slow_thr) ? v2 - 1 : v2;
    const int nx = x + v3;
    sumv += v3;
    if (nx < llen) {
      const uint32_t nw = pack_xvf(nx, v3, fl);
      if (j >= c0l) {  // an arrival: its whole record
        hot[G.sl[c]] = (v2u){nw, hw.y};
        cold[G.sl[c]] = cw;
      } else {
        hot_w[2 * G.sl[c]] = nw;
      }
      const int lcnt = s_pre[li + 1] - s_pre[li];
      if (j == 0) {
        s_ends[li].x = (int)nw;
        s_ends[li].y = cw.y;
      } else if (j == 1) {
        s_second[li] = make_int2((int)nw, cw.y);
      }
      if (j == lcnt - 1) s_ends[li].z = (int)nw;
    } else {  // only a lead vehicle of the previous step passes the node
      const int rp = cw.x;
      exit_t[rp] = cx.t;
      s_left[li] = 1;
      if (fl & kFlLast) {
        ++exits;
      } else {
        const uint32_t nfl = rinfo_flags((uint32_t)cw.y);
        const int tg = s_tgt[li];
        hb_out[tg] = (nfl & kFlLast) ? 0 : (int)route_info[rp + 2];
        ha_out[tg] = (v4i){cx.t, (int)pack_xvf(nx - llen, v3, nfl),
                           (int)hw.y, rp + 1};
        ht_out[tg] = (cx.t << 1) | (nx == llen ? 1 : 0);
        ++cross;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One kernel per step (see layout.h for when this is exact).  A wavefront
// takes a tile, one lane per thread, and performs the whole step on it:
//   1. merges the vehicle handed over to each lane in the previous step and
//      lets the head of each link's parking queue enter the lowest lane
//      whose cell 0 is empty (the arrivals join at the rear, in LDS);
//   2. decides each lead vehicle near the node: trip end (extra = vmax), or
//      the claim on its target lane that the previous step registered --
//      the smallest (rank, lane) key wins -- and, for the winner, the rear
//      of the target lane after that lane's own step-1 arrivals, recomputed
//      from the target link's previous state by the same rule;
//   3. moves every vehicle (second sub-step), rear first, 64 at a time;
//   4. writes the lanes' state for the next step and registers the claims
//      of the lanes' new lead vehicles for the next step.
template <bool kBatched>
__global__ __launch_bounds__(kWave) void k_step(
    const DevScen* __restrict__ descs, int slot, const int4* __restrict__ work,
    int step) {
  __shared__ int s_pre[kMaxTileLanes + 1];
  __shared__ int s_base[kMaxTileLanes], s_hp[kMaxTileLanes],
      s_len[kMaxTileLanes], s_cnt0[kMaxTileLanes], s_tgt[kMaxTileLanes],
      s_extra[kMaxTileLanes], s_left[kMaxTileLanes];
  __shared__ int4 s_ends[kMaxTileLanes];    // new lead xvf/ninfo, rear xvf
  __shared__ int2 s_second[kMaxTileLanes];  // the vehicle behind the lead
  __shared__ uint2 s_nhot[kMaxTileLanes][2];  // arrivals of this step
  __shared__ int2 s_ncold[kMaxTileLanes][2];
  __shared__ int4 s_plans[kMaxPlans];
  const long long c0 = wall_clock64();
  const int4 w = work[blockIdx.x];
  const DevScen& S = descs[kBatched ? w.x : slot];
  const int t = S.t + step;
  const int p = t & 1;
  const long long Q = S.n_lanes;
  const int vmax = S.vmax;
  const uint32_t key0 = S.key0, key1 = S.key1;
  const uint64_t slow_thr = S.slow_thr;
  const GAS v4i* __restrict__ ls_cur = gpv<v4i>(S.lane_state + p * Q);
  GAS v4i* __restrict__ ls_nxt = gpv<v4i>(S.lane_state + (p ^ 1) * Q);
  const GAS v4i* __restrict__ ha_in = gpv<v4i>(S.hand_a + (p ^ 1) * Q);
  const GAS int32_t* __restrict__ hb_in = gp(S.hand_b + (p ^ 1) * Q);
  GAS v4i* __restrict__ ha_out = gpv<v4i>(S.hand_a + p * Q);
  GAS int32_t* __restrict__ hb_out = gp(S.hand_b + p * Q);
  GAS int32_t* __restrict__ cl_cur = gp(S.claim + p * Q);
  GAS int32_t* __restrict__ cl_nxt = gp(S.claim + (p ^ 1) * Q);
  const GAS int32_t* __restrict__ qn_cur = gp(S.qnext + p * Q);
  GAS int32_t* __restrict__ qn_nxt = gp(S.qnext + (p ^ 1) * Q);
  const GAS int32_t* __restrict__ ht_in = gp(S.hand_tag + (p ^ 1) * Q);
  const GAS v2i* __restrict__ lane_bm = gpv<v2i>(S.lane_bm);
  const GAS int32_t* __restrict__ lane_qend = gp(S.lane_qend);
  GAS int32_t* __restrict__ ht_out = gp(S.hand_tag + p * Q);
  GAS int32_t* __restrict__ lane_qhead = gp(S.lane_qhead);
  GAS v4i* __restrict__ lane_qrec = gpv<v4i>(S.lane_qrec);
  const GAS v4i* __restrict__ wait_rec = gpv<v4i>(S.wait_rec);
  // hot and hot_w name the same records (loads / xvf stores): no restrict
  GAS v2u* hot = gpv<v2u>(S.hot);
  GAS uint32_t* hot_w = gpv<uint32_t>(S.hot);
  GAS v2i* cold = gpv<v2i>(S.cold);
  const GAS uint32_t* __restrict__ route_info = gp(S.route_info);
  GAS int32_t* __restrict__ exit_t = gp(S.exit_t);
  const int i = threadIdx.x;
  const int nl = w.z;
  const bool act = i < nl;
  const int g = w.y + i;

  // 1. what every lane needs from the previous step, in one round: its
  // static word, its state, the tag of the last handoff into it and (lane
  // 0) the departure time of its link's queue head
  // (threads past the tile's lanes read its first lane and drop it, so
  // that no load waits behind a branch)
  const int gg = act ? g : w.y;
  v2i bm = lane_bm[gg];
  v4i st = ls_cur[gg];
  int htag = ht_in[gg], qn = qn_cur[gg];
  if (!act) {
    bm = (v2i){0, 0};
    st = (v4i){0, 0, 0, 0};
    htag = kTagNone;
    qn = INT32_MAX;
  }
  load_plans(S, s_plans);
  const uint32_t meta = (uint32_t)bm.y;
  const int len = act ? lmeta_len(meta) : 1;
  const int k = lmeta_k(meta), lanes = lmeta_lanes(meta);
  const int key = lmeta_rank(meta) * 8 + k;
  const int head = hc_head(st.w);
  const int cnt = act ? hc_cnt(st.w) : 0;
  const uint32_t lead_w = (uint32_t)st.x;
  // a vehicle handed over in the previous step joins at the rear (its
  // record is read below); the tag says whether it landed on cell 0
  bool arr = false;
  if (act && (htag >> 1) == t - 1) {
    if (cnt >= len) atomicOr(S.err, SIM_DEVERR_LANE_FULL);
    else arr = true;
  }
  const int rear_x =
      arr ? ((htag & 1) ? 0 : 1) : (cnt > 0 ? xvf_x((uint32_t)st.z) : 1);
  const bool empty0 = act && rear_x != 0;
  const unsigned long long free0 = __ballot(empty0);
  const int l0 = i - k;  // this link's lane 0 in the tile
  const int qn0 = __shfl(qn, l0);
  int ins = 0;
  if (empty0) {
    const unsigned long long lm = (free0 >> l0) & ((1ull << lanes) - 1ull);
    if (__builtin_ctzll(lm) == k && qn0 <= t) ins = 1;
  }
  const unsigned long long insm = __ballot(ins);
  const bool link_ins =
      act && k == 0 && ((insm >> i) & ((1ull << lanes) - 1ull)) != 0;
  const int n_new = (arr ? 1 : 0) + ins;
  // second round, only where something arrives: the handed-over record,
  // and the head of the parking queue (read by lane 0, which also
  // prefetches the next head for the next step)
  v4i ha = {0, 0, 0, 0}, qrec = {0, 0, 0, 0}, nrec = {-1, 0, 0, 0};
  int hb = 0, qh = 0, qend = 0;
  if (arr) {
    ha = ha_in[g];
    hb = hb_in[g];
  }
  if (link_ins) {
    qh = lane_qhead[g];
    qrec = lane_qrec[g];
    qend = lane_qend[g];
  }

  // 2. the lead vehicle at the node: target lane, its claim, and the
  // arrivals of the target link's lanes (read by every candidate, used by
  // the winner)
  // (a red light holds it back: no claim, no trip end)
  wave_lds_sync();  // the plans in LDS
  const bool cand = act && cnt > 0 && len - 1 - xvf_x(lead_w) < vmax &&
                    !sig_red(s_plans, meta, t);
  const bool exits_here = cand && (xvf_fl(lead_w) & kFlLast);
  int tgt = exits_here ? -2 : -1, tm = 0, tlanes = 1, tl0 = 0;
  int claim = INT32_MAX, tqn = INT32_MAX;
  int trear[4], tpend[4], tcnt[4];
  if (cand && !exits_here) {
    const uint32_t ni = (uint32_t)st.y;
    tl0 = rinfo_lane0(ni);
    tlanes = rinfo_lanes(ni);
    tm = min(k, tlanes - 1);
    tgt = tl0 + tm;
    claim = cl_cur[tgt];
    tqn = qn_cur[tl0];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    trear[m] = 0;
    tpend[m] = kTagNone;
    tcnt[m] = 0;
    if (tgt >= 0 && m < tlanes) {
      const v4i ts = ls_cur[tl0 + m];
      const v4i th = ha_in[tl0 + m];
      trear[m] = (int)ts.z;
      tcnt[m] = hc_cnt(ts.w);
      tpend[m] = th.x == t - 1 ? th.y : kTagNone;
    }
  }
  if (act) {
    s_base[i] = bm.x;
    s_hp[i] = hc_make(head, 0, 0);
    s_len[i] = len;
    s_cnt0[i] = cnt;
    s_tgt[i] = tgt;
    s_left[i] = 0;
    s_ends[i] = make_int4(0, 0, 0, 0);
  }
  const int cntn = cnt + n_new;
  int incl = cntn;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (i >= off) incl += y;
  }
  const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1));
  if (i < nl) s_pre[i] = incl - cntn;
  if (i == 0) s_pre[nl] = total;
  const unsigned long long cocc =
      wave_sum((unsigned long long)(cntn > 0 ? len : 0));
  wave_lds_sync();

  // 3. the move, groups of kGroup x 64 vehicles from the rear: a group
  // loads every record it needs before it rewrites any, so each vehicle
  // reads the position of the one ahead before that one moves
  unsigned long long sumv = 0, cross = 0, exits = 0;
  const int nchunk = (total + kWave - 1) / kWave;
  const StepCtx cx{t, vmax, key0, key1, slow_thr};
  bool first = true;
  // (one pass with no vehicle still decides the winners)
  for (int gr = ((nchunk - 1) / kGroup) * kGroup; gr >= 0; gr -= kGroup) {
    StepGroup G;
    step_load(G, gr, i, total, nl, s_pre, s_len, s_base, s_hp, hot, hot_w,
              cold);
    if (first) {
      first = false;
      // the arrivals' records go to LDS; the inserting lane takes the queue
      // head that lane 0 of its link read
      const int qid = __shfl(qrec.x, l0), qdep = __shfl(qrec.y, l0),
                qrp = __shfl(qrec.z, l0), qni = __shfl(qrec.w, l0);
      if (arr) {
        s_nhot[i][0] = make_uint2((uint32_t)ha.y, (uint32_t)ha.z);
        s_ncold[i][0] = make_int2(ha.w, hb);
      }
      if (ins) {
        s_nhot[i][arr ? 1 : 0] = make_uint2(
            pack_xvf(0, 0, (uint32_t)qdep >> kDepartBits), (uint32_t)qid);
        s_ncold[i][arr ? 1 : 0] = make_int2(qrp, qni);
      }
      if (link_ins && qh + 1 < qend) nrec = wait_rec[qh + 1];
      // winners: extra cells past the link end (rule R7); the claim is
      // cleared for the next use of this buffer
      if (act) {
        int extra = exits_here ? vmax : 0;
        if (tgt >= 0 && claim == key) {
          cl_cur[tgt] = INT32_MAX;
          // the target link's step-1 arrivals, by the rule of part 1
          int rx[4];
          unsigned free_m = 0;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            rx[m] = tpend[m] != kTagNone ? xvf_x((uint32_t)tpend[m])
                    : tcnt[m] > 0         ? xvf_x((uint32_t)trear[m])
                                          : vmax;
            if (m < tlanes && rx[m] != 0) free_m |= 1u << m;
          }
          const bool tins =
              tqn <= t && free_m != 0 && __builtin_ctz(free_m) == tm;
          extra = tins ? 0 : min(vmax, rx[tm]);
        }
        s_extra[i] = extra;
      }
      wave_lds_sync();
    }
    step_run(G, cx, s_len, s_cnt0, s_pre, s_extra, s_tgt, s_nhot, s_ncold,
             s_ends, s_second, s_left, hot, hot_w, cold, route_info, exit_t,
             ha_out, hb_out, ht_out, sumv, cross, exits);
  }
  wave_lds_sync();

  // 4. the lanes for the next step, and the claims of their new leads
  if (act) {
    int4 e = s_ends[i];
    int h1 = head, c1 = cntn;
    if (s_left[i]) {
      h1 = wrapi(head + 1, len);
      c1 = cntn - 1;
      const int2 sec = s_second[i];
      e.x = sec.x;  // the vehicle behind is the new lead
      e.y = sec.y;
    }
    ls_nxt[g] = (v4i){e.x, e.y, e.z, hc_make(h1, 0, c1)};
    if (c1 > 0 && len - 1 - xvf_x((uint32_t)e.x) < vmax &&
        !(xvf_fl((uint32_t)e.x) & kFlLast) && !sig_red(s_plans, meta, t + 1)) {
      const uint32_t ni = (uint32_t)e.y;
      atomicMin((int*)&cl_nxt[rinfo_lane0(ni) + min(k, rinfo_lanes(ni) - 1)],
                key);
    }
    if (k == 0) {
      if (link_ins) {
        lane_qhead[g] = qh + 1;
        lane_qrec[g] = nrec;
        qn_nxt[g] = qh + 1 < qend ? (nrec.y & ((1 << kDepartBits) - 1))
                                  : INT32_MAX;
      } else {
        qn_nxt[g] = qn;
      }
    }
  }
  sumv = wave_sum(sumv);
  cross = wave_sum(cross);
  exits = wave_sum(exits);
  const unsigned long long n_ins = wave_sum((unsigned long long)ins);
  if (i == 0) {
    GAS unsigned long long* ctr =
        (GAS unsigned long long*)gp(S.tile_ctr + (long long)w.y * C_N);
    atomicAdd((unsigned long long*)&ctr[C_UPDATES], (unsigned long long)total);
    atomicAdd((unsigned long long*)&ctr[C_SUMV], sumv);
    if (cross) atomicAdd((unsigned long long*)&ctr[C_CROSS], cross);
    if (exits) atomicAdd((unsigned long long*)&ctr[C_EXITS], exits);
    if (n_ins) atomicAdd((unsigned long long*)&ctr[C_INS], n_ins);
    atomicAdd((unsigned long long*)&ctr[C_COCC], cocc);
    atomicAdd((unsigned long long*)&ctr[C_CYCLES],
              (unsigned long long)(wall_clock64() - c0));
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

// ---- launchers -------------------------------------------------------------

hipError_t launch_front(const DevScen* d_descs, int slot, const int4* d_work,
                        int n_work, int pieces, int step, int lc_words,
                        hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  if (slot < 0)
    hipLaunchKernelGGL(k_front<true>, dim3(n_work), dim3(kWave),
                       (size_t)kLcBytesPerWord * lc_words, s, d_descs, 0, d_work, 1, step);
  else
    hipLaunchKernelGGL(k_front<false>, dim3(n_work), dim3(kWave),
                       (size_t)kLcBytesPerWord * lc_words, s, d_descs, slot, d_work, pieces,
                       step);
  return hipGetLastError();
}

hipError_t launch_back(const DevScen* d_descs, int slot, const int4* d_work,
                       int n_work, int n_extra, int step, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  if (slot < 0)
    hipLaunchKernelGGL(k_back<true>, dim3(n_work), dim3(kWave), 0, s, d_descs,
                       0, d_work, n_work, step);
  else
    hipLaunchKernelGGL(k_back<false>, dim3(n_work + n_extra), dim3(kWave), 0,
                       s, d_descs, slot, d_work, n_work, step);
  return hipGetLastError();
}

hipError_t launch_step(const DevScen* d_descs, int slot, const int4* d_work,
                       int n_work, int step, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  if (slot < 0)
    hipLaunchKernelGGL(k_step<true>, dim3(n_work), dim3(kWave), 0, s, d_descs,
                       0, d_work, step);
  else
    hipLaunchKernelGGL(k_step<false>, dim3(n_work), dim3(kWave), 0, s,
                       d_descs, slot, d_work, step);
  return hipGetLastError();
}

void* step_kernel(bool batched) {
  return batched ? reinterpret_cast<void*>(&k_step<true>)
                 : reinterpret_cast<void*>(&k_step<false>);
}

void* front_kernel(bool batched) {
  return batched ? reinterpret_cast<void*>(&k_front<true>)
                 : reinterpret_cast<void*>(&k_front<false>);
}
void* back_kernel(bool batched) {
  return batched ? reinterpret_cast<void*>(&k_back<true>)
                 : reinterpret_cast<void*>(&k_back<false>);
}
void* advance_kernel() { return reinterpret_cast<void*>(&k_advance); }

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
                         int n_links, int n_lanes, int ring, hipStream_t s) {
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
