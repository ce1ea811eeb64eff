// front_back.hip -- the two-kernel form of the TRANSIMS per-second update
// (gfx950), used with lane changes or short links.
//
// A step is two kernels, the GPU form of the paper's per-step sequence of a
// lane-change sub-step and a velocity-and-move sub-step, each followed by a
// boundary exchange (Section "Micro-simulation parallelization: Domain
// decomposition"): the kernel boundaries are the two exchanges.  Each
// workgroup is one wavefront that owns a tile of whole links (at most 64
// lanes); a lane's vehicles live in a lead-first ring buffer, so the
// per-step traffic is proportional to the vehicles, not to the cells.
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
#include "device.h"
#include "kernels.h"
#include "philox.h"
#include "transims.h"

namespace tr {

namespace {

// load of a lane in the move sub-step: its vehicles plus a fixed cost; a
// tile gets one move wavefront per kPieceCost of load (up to a limit)
constexpr int kLaneCost = 4;
constexpr int kPieceCost = 512;

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
// The scenario's lane-change parameters, read from the descriptor once per
// tile (uniform values, kept in scalar registers)
struct LcParams {
  int vmax, desp;
  uint64_t thr;
  uint32_t key0, key1;
};

__device__ int lc_decide(const LcParams& P, const uint32_t* wk, int wpl,
                         int len, int lanes, int k, int x, int v, uint32_t fl,
                         int id, int t) {
  const int vmax = P.vmax;
  const int lo = fl_lo(fl), hi = fl_hi(fl);
  if (k < lo || k > hi) {  // mandatory: one lane toward the turn lanes
    const int m = k < lo ? k + 1 : k - 1;
    const uint32_t* wm = wk + (m - k) * wpl;
    const int need = min(vmax, (len - 1 - x) / P.desp);
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
  // a threshold of 2^32 takes every draw, which is then not made
  if (P.thr < (1ull << 32) &&
      (uint64_t)veh_draw((uint32_t)id, (uint32_t)t, 0u, P.key0, P.key1) >=
          P.thr)
    return -1;
  return best;
}

// Largest j < n with pre[j] <= f (pre ascending, pre[0] = 0 <= f, n at
// most kMaxTileLanes), with pre[j] in *pj.  The steps are the fixed powers
// of two below kMaxTileLanes, taken with no branch at all, so the compiler
// overlaps the searches of a thread's several vehicles instead of running
// one search after another.
__device__ __forceinline__ int lc_find(const int* pre, int n, int f,
                                       int* pj = nullptr) {
  int lo = 0, plo = 0;
#pragma unroll
  for (int s = kMaxTileLanes / 2; s >= 1; s >>= 1) {
    const int j = min(lo + s, n - 1);
    const int pv = pre[j];
    const bool up = pv <= f;
    lo = up ? j : lo;
    plo = up ? pv : plo;
  }
  if (pj) *pj = plo;
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

// What a lane thread (thread j < nl) holds of lane j for finding records:
// the lane's first vehicle in the tile's numbering, the start of its
// current ring half, and its ring head | length << 16.
struct LcLane {
  int vp, org, hl;
};

// Lane and record slot of vehicle f of the tile's numbering (lanes in
// order, each lane lead first), for F <= f <= Fl < F + kWave with F and Fl
// the same in every thread; called by the whole wave.  The lanes that hold
// vehicles F to Fl follow from two ballots over the lane threads' first
// vehicles; each thread then counts the lanes of that range that start at
// or before its vehicle, and takes the ring position from the lane
// thread's registers.
__device__ __forceinline__ void lc_locate(const LcLane& R, int nl, int F,
                                          int Fl, int f, int& ln, int& slot) {
  const bool lt = (int)threadIdx.x < nl;
  const int l0 = __popcll(__ballot(lt && R.vp <= F)) - 1;
  const int l1 = __popcll(__ballot(lt && R.vp <= Fl)) - 1;
  int vp, org, hl;
  if (l1 == l0) {  // one lane holds the whole batch
    ln = l0;
    vp = __builtin_amdgcn_readlane(R.vp, l0);
    org = __builtin_amdgcn_readlane(R.org, l0);
    hl = __builtin_amdgcn_readlane(R.hl, l0);
  } else {
    int l = l0;
    for (int j = l0 + 1; j <= l1; ++j)
      l += __builtin_amdgcn_readlane(R.vp, j) <= f ? 1 : 0;
    ln = l;
    vp = __shfl(R.vp, l);
    org = __shfl(R.org, l);
    hl = __shfl(R.hl, l);
  }
  slot = org + wrapi((hl & 0xFFFF) + f - vp, hl >> 16);
}

// Vehicles per thread whose records stay in registers through the
// sub-step (the tile's first kLcRes * kWave vehicles: one round of loads);
// the rest are loaded again by each phase, a batch per thread at a time
// (a jammed tile holds thousands of vehicles, and each batch costs one
// round trip to memory, so the phases with few live values per vehicle
// take wider batches).
constexpr int kLcRes = 2;
constexpr int kLcOccBatch = 6;    // occupancy: the xvf word
constexpr int kLcDecBatch = 4;    // decisions: the hot record
constexpr int kLcPlaceBatch = 6;  // placement: hot and cold records

__device__ __forceinline__ void lc_mark_occ(const LcTile& T, const LcLat& Z,
                                            int ln, uint32_t xw) {
  const int x = xvf_x(xw);
  atomicOr(&Z.occ[T.wo[ln] + (x >> 5)], 1u << (x & 31));
}

__device__ __forceinline__ void lc_mark_move(const LcParams& P, const LcTile& T,
                                             const LcLat& Z, int t, int ln,
                                             v2u hw) {
  const uint32_t meta = (uint32_t)T.info[ln].y;
  const int len = lmeta_len(meta), k = lmeta_k(meta);
  const int wl = (len + 31) >> 5, q0 = T.wo[ln];
  const int x = xvf_x(hw.x);
  const int d = lc_decide(P, Z.occ + q0, wl, len, lmeta_lanes(meta), k, x,
                          xvf_v(hw.x), xvf_fl(hw.x), (int)hw.y, t);
  if (d < 0) return;
  atomicOr(d > k ? &Z.rgt[q0 + (x >> 5)] : &Z.lft[q0 + (x >> 5)],
           1u << (x & 31));
}

// Writes the vehicle's records at its place in its lane after the sub-step
// (links with a move only).
__device__ __forceinline__ void lc_place(GAS v2u* hot, GAS v2i* cold,
                                         uint32_t* err, const LcTile& T,
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
    atomicOr(err, SIM_DEVERR_LANE_FULL);
    return;
  }
  const int npar = 1 - hc_par(T.hp[ln]);
  const int dst = T.info[lnd].x + npar * len + j;
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
  uint32_t* const err = S.err;
  const LcParams P{S.vmax, S.lc_desp, S.lc_thr, S.key0, S.key1};
  int wpl = 0, nv = 0, k = 0;
  if (i < nl) {
    const uint32_t meta = (uint32_t)T.info[i].y;
    if (lmeta_lanes(meta) >= 2) {
      wpl = (lmeta_len(meta) + 31) >> 5;
      nv = T.cnt[i];
      k = lmeta_k(meta);
    }
  }
  const int wi = wave_scan(wpl), vi = wave_scan(nv);
  const int Wt = wave_last(wi), V = wave_last(vi);
  if (V == 0) return 0;
  LcLane R{0, 0, 0};
  if (i < nl) {
    T.wo[i] = wi - wpl;
    T.vp[i] = vi - nv;
    T.mv[i] = 0;
    const int len = lmeta_len((uint32_t)T.info[i].y), hp = T.hp[i];
    R = LcLane{vi - nv, T.info[i].x + hc_par(hp) * len,
               hc_head(hp) | (len << 16)};
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
      lc_locate(R, nl, min(u * kWave, V - 1), min(u * kWave + kWave, V) - 1,
                min(u * kWave + i, V - 1), rln[u], rsl[u]);
#pragma unroll
    for (int u = 0; u < kLcRes; ++u) {
      rhw[u] = hot[rsl[u]];
      rcw[u] = cold[rsl[u]];
    }
  }
  const int f_rest = kLcRes * kWave;  // first vehicle of the loops below

  // A vehicle can only change lanes if it must (it is outside the lanes of
  // its next turn) or if its own lane holds it back: fewer than
  // min(v+1, vmax) empty cells ahead.  Both follow from its record and the
  // record ahead of it in its lane (the tile's vehicles are numbered lane by
  // lane, lead first), so when no vehicle of the tile qualifies the sub-step
  // changes nothing and the lattice is never built.  Vehicles past the
  // first kLcRes * kWave count as qualifying.
  {
    const int vmax = P.vmax;
    bool want = V > f_rest;
    int prev_x = 0;
#pragma unroll
    for (int u = 0; u < kLcRes; ++u) {
      const int f = u * kWave + i;
      const int x = xvf_x(rhw[u].x);
      const int px = wave_prev(x, u > 0 ? wave_last(prev_x) : 0);
      prev_x = x;
      if (f < V) {
        const uint32_t meta = (uint32_t)T.info[rln[u]].y;
        const uint32_t fl = xvf_fl(rhw[u].x);
        const int k = lmeta_k(meta), len = lmeta_len(meta);
        const bool lead = f == T.vp[rln[u]];
        const int own = min(vmax, lead ? len - 1 - x : px - x - 1);
        if (k < fl_lo(fl) || k > fl_hi(fl) ||
            own < min(xvf_v(rhw[u].x) + 1, vmax))
          want = true;
      }
    }
    if (__ballot(want) == 0ull) return 0;
  }
  for (int q = i; q < Wt; q += kWave) {
    Z.occ[q] = 0u;
    Z.rgt[q] = 0u;
    Z.lft[q] = 0u;
  }
  __syncthreads();

  // occupancy.  The first reload batch keeps its vehicles' lanes and xvf
  // words in registers for the decisions, which need nothing else of a
  // vehicle when no draw is taken (a lane-change threshold of 2^32).
#pragma unroll
  for (int u = 0; u < kLcRes; ++u)
    if (u * kWave + i < V) lc_mark_occ(T, Z, rln[u], rhw[u].x);
  const bool keep = P.thr >= (1ull << 32);
  int kln[kLcOccBatch];
  uint32_t kxw[kLcOccBatch];
  if (V > f_rest) {
    int sl[kLcOccBatch];
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u)
      lc_locate(R, nl, min(f_rest + u * kWave, V - 1),
                min(f_rest + u * kWave + kWave, V) - 1,
                min(f_rest + u * kWave + i, V - 1), kln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u) kxw[u] = hot[sl[u]].x;
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u)
      if (f_rest + u * kWave + i < V) lc_mark_occ(T, Z, kln[u], kxw[u]);
  }
  for (int f0 = f_rest + kLcOccBatch * kWave; f0 < V;
       f0 += kLcOccBatch * kWave) {
    int ln[kLcOccBatch], sl[kLcOccBatch];
    uint32_t xw[kLcOccBatch];
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u)
      lc_locate(R, nl, min(f0 + u * kWave, V - 1),
                min(f0 + u * kWave + kWave, V) - 1,
                min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u) xw[u] = hot[sl[u]].x;
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u)
      if (f0 + u * kWave + i < V) lc_mark_occ(T, Z, ln[u], xw[u]);
  }
  __syncthreads();

  // decisions
#pragma unroll
  for (int u = 0; u < kLcRes; ++u)
    if (u * kWave + i < V) lc_mark_move(P, T, Z, t, rln[u], rhw[u]);
  int f_dec = f_rest;  // first vehicle the loop below reloads
  if (keep && V > f_rest) {
#pragma unroll
    for (int u = 0; u < kLcOccBatch; ++u)
      if (f_rest + u * kWave + i < V)
        lc_mark_move(P, T, Z, t, kln[u], (v2u){kxw[u], 0u});
    f_dec = f_rest + kLcOccBatch * kWave;
  }
  for (int f0 = f_dec; f0 < V; f0 += kLcDecBatch * kWave) {
    int ln[kLcDecBatch], sl[kLcDecBatch];
    v2u hw[kLcDecBatch];
#pragma unroll
    for (int u = 0; u < kLcDecBatch; ++u)
      lc_locate(R, nl, min(f0 + u * kWave, V - 1),
                min(f0 + u * kWave + kWave, V) - 1,
                min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcDecBatch; ++u) hw[u] = hot[sl[u]];
#pragma unroll
    for (int u = 0; u < kLcDecBatch; ++u)
      if (f0 + u * kWave + i < V) lc_mark_move(P, T, Z, t, ln[u], hw[u]);
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
  moved = (int)wave_sum(moved);
  if (moved == 0) return 0;
  int carry = 0;
  for (int q0 = 0; q0 < Wt; q0 += kWave) {
    const int q = q0 + i;
    const int c = wave_scan(q < Wt ? __popc(Z.occ[q]) : 0);
    if (q < Wt) Z.pre[q] = (uint16_t)(carry + c);
    carry += wave_last(c);
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
    if (u * kWave + i < V)
      lc_place(hot, cold, err, T, Z, rln[u], rhw[u], rcw[u]);
  for (int f0 = f_rest; f0 < V; f0 += kLcPlaceBatch * kWave) {
    int ln[kLcPlaceBatch], sl[kLcPlaceBatch];
    v2u hw[kLcPlaceBatch];
    v2i cw[kLcPlaceBatch];
#pragma unroll
    for (int u = 0; u < kLcPlaceBatch; ++u)
      lc_locate(R, nl, min(f0 + u * kWave, V - 1),
                min(f0 + u * kWave + kWave, V) - 1,
                min(f0 + u * kWave + i, V - 1), ln[u], sl[u]);
#pragma unroll
    for (int u = 0; u < kLcPlaceBatch; ++u) {
      hw[u] = hot[sl[u]];
      cw[u] = cold[sl[u]];
    }
#pragma unroll
    for (int u = 0; u < kLcPlaceBatch; ++u)
      if (f0 + u * kWave + i < V)
        lc_place(hot, cold, err, T, Z, ln[u], hw[u], cw[u]);
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
  // what the end of the kernel writes through, read with the rest of the
  // descriptor rather than one field after another at the end
  const int xcap = S.xcap;
  int* const xcount = S.xcount;
  int4* const xlist = S.xlist;
  int* const tile_np = S.tile_np;
  long long* const ftile_ctr = S.ftile_ctr;
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
  if (pieces > 1 && xcap > 0) {
    const unsigned long long T =
        wave_sum(act ? cnt + kLaneCost : 0);
    const int np = min(pieces, (int)((T + kPieceCost - 1) / kPieceCost));
    if (i == 0) {
      int got = 0;
      if (np > 1) {
        const int xb = atomicAdd(&xcount[t & 1], np - 1);
        got = max(0, min(xcap - xb, np - 1));
        for (int r = 0; r < got; ++r)
          xlist[xb + r] =
              make_int4(w.y, w.z | ((r + 1) << 8) | ((got + 1) << 16), w.w, 0);
      }
      tile_np[w.w] = got + 1;
    }
  }
  const unsigned long long n_ins = wave_sum(ins);
  if (i == 0) {
    long long* ctr = ftile_ctr + (long long)w.w * C_N;
    if (n_ins) atomicAdd((unsigned long long*)&ctr[C_INS], n_ins);
    if (lc_moves) atomicAdd((unsigned long long*)&ctr[C_LC],
                            (unsigned long long)lc_moves);
    atomicAdd((unsigned long long*)&ctr[C_CYCLES],
              (unsigned long long)(wall_clock64() - c0));
  }
}

// The back kernel: one wavefront per tile of at most 64 lanes, plus the
// extra wavefronts the front kernel listed for heavy tiles.  The wavefronts
// of a tile cut it into as many contiguous runs of lanes of about equal load
// (vehicles + kLaneCost per lane) -- the paper's load balancing by measured
// load, redone every step from the current counts -- and each takes one run.
// Lane threads resolve the intersections, then the vehicles of the run are
// updated 64 at a time.

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
  // A single slot's extra wavefronts of heavy tiles take the first xcap
  // blocks, so that they start with the first tiles (the heaviest, in a
  // list ordered by measured time) instead of after every tile; the tiles
  // follow, xcap (a multiple of 8) keeping each on its XCD.
  const int xcap = kBatched ? 0 : descs[slot].xcap;
  int4 w;
  int piece = 0, np = 1;
  if ((int)blockIdx.x >= xcap) {
    w = work[blockIdx.x - xcap];
    if (xcap > 0) np = descs[slot].tile_np[w.w];
  } else {  // an extra wavefront of a heavy tile (single slot only)
    const DevScen& S1 = descs[slot];
    const int e = (int)blockIdx.x;
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
    const int ci = wave_scan(cost);
    const int T = wave_last(ci);
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
  const int incl = wave_scan(cnt);
  const int total = wave_last(incl);  // in a scalar register
  // every lane of the tile gets its entry (lanes outside the run hold no
  // vehicles of it), so the search below only ever lands on the run's lanes
  if (i < nl) s_pre[i] = incl - cnt;
  if (i == 0) s_pre[nl] = total;
  const unsigned long long cocc =
      wave_sum(cnt > 0 ? len : 0);
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
        const int fr0 = (g0 + c) * kWave, fr = fr0 + i;
        const int f = min(fr, total - 1);
        const int lo = wave_lane_of(incl - cnt, nl, min(fr0, total - 1),
                                    min(fr0 + kWave - 1, total - 1), f);
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
  sumv = wave_sum((int)sumv);
  cross = wave_sum((int)cross);
  exits = wave_sum((int)exits);
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

// ---- launchers -------------------------------------------------------------

// Each launcher first clears any error left by earlier runtime calls of this
// thread, so that the status it returns is the launch's own.
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

void* front_kernel(bool batched) {
  return batched ? reinterpret_cast<void*>(&k_front<true>)
                 : reinterpret_cast<void*>(&k_front<false>);
}
void* back_kernel(bool batched) {
  return batched ? reinterpret_cast<void*>(&k_back<true>)
                 : reinterpret_cast<void*>(&k_back<false>);
}

}  // namespace tr
