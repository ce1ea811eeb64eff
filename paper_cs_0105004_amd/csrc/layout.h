// layout.h -- device-resident state of one scenario slot, shared by the host
// side of libtransims and its kernels.
//
// Vehicles are stored per lane as an ordered queue (lead first) in a ring
// buffer with one record slot per cell of the lane: vehicles never overtake
// inside a lane, so the order only changes when a vehicle enters at the rear
// (parking, arrival from an upstream node, lane change) or leaves at the
// front (next link, trip end) -- or moves sideways.  A record is
//   hot  = { xvf, id }     8 bytes, read and its xvf word rewritten every step
//   cold = { rp, ninfo }   8 bytes, read only when the vehicle nears a node
// xvf packs x (bits 0-15), v (bits 16-19) and flags (bits 20-24: last link;
// lowest and highest lane from which the next turn is made).  rp is the
// vehicle's absolute route index; ninfo is the route info word of the next
// route entry (see below), so the lane it aims at needs no further lookup.
//
// Route info word (one per route entry r, replacing the link id):
//   bits 0-23 first lane id of link route[r]; 24-25 lanes-1;
//   26-27 / 28-29 lowest / highest lane of route[r] from which the turn into
//   route[r+1] is made; 30 r is the last entry of the route.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tr {

constexpr int kWave = 64;
constexpr int kMaxTileLanes = 64;
constexpr int32_t kTagNone = INT32_MIN;
constexpr int kRingMax = 4096;  // vehicles of one ring scenario (kept in LDS)

__host__ __device__ inline uint32_t pack_xvf(int x, int v, uint32_t fl) {
  return (uint32_t)x | ((uint32_t)v << 16) | (fl << 20);
}
__host__ __device__ inline int xvf_x(uint32_t w) { return (int)(w & 0xFFFFu); }
__host__ __device__ inline int xvf_v(uint32_t w) {
  return (int)((w >> 16) & 0xFu);
}
__host__ __device__ inline uint32_t xvf_fl(uint32_t w) { return w >> 20; }

constexpr uint32_t kFlLast = 1u;

__host__ __device__ inline uint32_t rinfo_make(int lane0, int lanes, int lo,
                                               int hi, bool last) {
  return (uint32_t)lane0 | ((uint32_t)(lanes - 1) << 24) |
         ((uint32_t)lo << 26) | ((uint32_t)hi << 28) |
         (last ? (1u << 30) : 0u);
}
__host__ __device__ inline int rinfo_lane0(uint32_t r) {
  return (int)(r & 0xFFFFFFu);
}
__host__ __device__ inline int rinfo_lanes(uint32_t r) {
  return (int)((r >> 24) & 3u) + 1;
}
// record flags of a vehicle on the link of route entry with info r
__host__ __device__ inline uint32_t rinfo_flags(uint32_t r) {
  return ((r >> 30) & 1u) | (((r >> 26) & 3u) << 1) | (((r >> 28) & 3u) << 3);
}

// a lane's queue: head index (bits 0-14), buffer parity (15), count (16-31)
__host__ __device__ inline int hc_make(int head, int par, int cnt) {
  return head | (par << 15) | (cnt << 16);
}
__host__ __device__ inline int hc_head(int h) { return h & 0x7FFF; }
__host__ __device__ inline int hc_par(int h) { return (h >> 15) & 1; }
__host__ __device__ inline int hc_cnt(int h) { return (int)((uint32_t)h >> 16); }

// a waiting vehicle: {id, depart | flags on its first link << 27, rp of its
// first route entry, route info of its second entry (0 if none)}
constexpr int kDepartBits = 27;

// static per-lane word: len (bits 0-14), lane index k (15-16), lanes-1
// (17-18), rank of the link at its downstream node (19-25), signal plan + 1
// of the link (26-31, 0 = unsignalised)
__host__ __device__ inline uint32_t lmeta_make(int len, int k, int lanes,
                                               int rank, int plan = -1) {
  return (uint32_t)len | ((uint32_t)k << 15) | ((uint32_t)(lanes - 1) << 17) |
         ((uint32_t)rank << 19) | ((uint32_t)(plan + 1) << 26);
}
__host__ __device__ inline int lmeta_plan(uint32_t m) {
  return (int)(m >> 26) - 1;
}
constexpr int kMaxPlans = 63;
__host__ __device__ inline int lmeta_len(uint32_t m) { return (int)(m & 0x7FFFu); }
__host__ __device__ inline int lmeta_k(uint32_t m) { return (int)((m >> 15) & 3u); }
__host__ __device__ inline int lmeta_lanes(uint32_t m) {
  return (int)((m >> 17) & 3u) + 1;
}
__host__ __device__ inline int lmeta_rank(uint32_t m) {
  return (int)((m >> 19) & 0x7Fu);
}
__host__ __device__ inline uint32_t fl_make(bool last, int lo, int hi) {
  return (last ? kFlLast : 0u) | ((uint32_t)lo << 1) | ((uint32_t)hi << 3);
}
__host__ __device__ inline int fl_lo(uint32_t fl) { return (fl >> 1) & 3; }
__host__ __device__ inline int fl_hi(uint32_t fl) { return (fl >> 3) & 3; }

// per-tile counters (int64), accumulated over steps
enum : int {
  C_UPDATES = 0,
  C_SUMV,
  C_CROSS,
  C_EXITS,
  C_LC,
  C_INS,
  C_COCC,
  C_CYCLES,
  C_N
};

// lane summary written by the front kernel for the back kernel, which never
// modifies it:
//   x = target lane id of the lead vehicle (-1: not near the node, -2: trip
//       ends at the node), y = x of the rearmost vehicle (len if empty),
//   z = the lane's queue (hc) as the move finds it

// One kernel per step.  Without lane changes, and with every link at least
// 2*vmax cells long, each input of a step that another tile produces is
// final when the previous step ends: the lead vehicles that compete at a
// node (a vehicle that arrives in a step lands within vmax-1 cells of the
// link start, so it cannot reach the node region in that step), their
// claims (made by the previous step's move), and the state of a target
// link's lanes and parking queue.  Those arrays are then kept twice and
// indexed by step parity: in step t a kernel reads buffer t&1 of lane_state,
// claim and qnext and buffer (t-1)&1 of the handoff slots, and writes the
// other one.  With `fused` == 0 only buffer 0 is used.

struct DevScen {
  // ---- what every step kernel reads first, kept contiguous so that it
  // arrives in one round of wide scalar loads ----
  int32_t t;  // index of the next step
  int32_t n_lanes;
  int32_t vmax;
  int32_t n_plans;
  // lanes: lane_bm {record base, lmeta}; lane_state[2][n_lanes] {lead xvf,
  // lead ninfo, rear xvf, hc} at the end of a step (one buffer without
  // fused stepping); hand_tag (fused) t << 1 | (landed on cell 0) of the
  // last handoff into the lane in a step of that parity; qnext (fused) the
  // departure of the link's parking-queue head (INT32_MAX: empty), at lane 0
  const int2* lane_bm;
  int4* lane_state;
  int32_t* hand_tag;
  int32_t* qnext;
  // fixed-time signal plans {cycle, red, offset, 0}: red at step t iff
  // (t + offset) % cycle < red
  const int4* plans;
  // one-kernel step, per tile and step parity: tile_live bit i = lane i of
  // the tile held a vehicle at the start of this step or of the step before
  // (so both parity buffers of a lane outside the mask hold its empty
  // state); tile_wake = the step from which the tile must look at every
  // lane (a parking-queue head may leave, or a queue moved on in the step
  // before).  arr_bits[parity][lane / 64]: bit set when a vehicle was handed
  // over into the lane in a step of that parity; cleared by the lane's
  // tile when it merges the vehicle.
  unsigned long long* tile_live;
  int32_t* tile_wake;
  unsigned long long* arr_bits;
  // arrival handoff per target lane: hand_a {tag = t, xvf, id, rp}, hand_b
  // ninfo
  int4* hand_a;
  int32_t* hand_b;
  int32_t* claim;  // smallest (rank, lane) key aiming at the lane
  // parking queue of a link, kept with its lane 0: the index of its head in
  // wait_rec and a copy of that record (id -1: to be fetched again), and
  // its end
  int32_t* lane_qhead;
  int4* lane_qrec;
  const int32_t* lane_qend;
  const int4* wait_rec;  // parking queues, link by link, by (depart, id)
  // vehicle records
  uint2* hot;
  int2* cold;
  // routes
  const uint32_t* route_info;
  int32_t* exit_t;
  long long* tile_ctr;  // [n_lanes * C_N], counters by a tile's first lane
  uint32_t* err;
  uint32_t key0, key1;  // Philox key = seed
  uint64_t slow_thr;
  // ---- the rest ----
  uint32_t flags;
  int32_t fused;  // 1: one kernel per step, parity-buffered state
  uint64_t lc_thr;
  int32_t lc_desp;
  int32_t n_links, n_tiles, n_ftiles, n_veh;
  int32_t ring_L, ring_n;
  int32_t lc_words;  // most lane-change lattice words of one tile
  int64_t n_route;
  const int32_t* link_ext;  // caller's link id, in the internal order
  // lanes: {record base, lmeta, link, end of the link's parking queue}
  const int4* lane_info;
  int4* lane_sum;  // two-kernel step: {target, rear x, hc, 0} after sub-step 1
  long long* ftile_ctr;  // [n_ftiles * C_N], front tiles
  // Heavy tiles get extra move wavefronts: the front kernel decides each
  // tile's number of runs (tile_np) and lists the runs beyond the first in
  // xlist {first lane, lanes | run << 8 | runs << 16, tile, 0}; xcount[t & 1]
  // counts them (reset one step ahead by the move kernel).
  int32_t* tile_np;
  int4* xlist;
  int32_t* xcount;
  int32_t xcap;  // entries of xlist (0: every tile is one run)
  const int64_t* route_off;
  // ring mode (vehicles in cyclic order)
  int32_t* ring_x;
  int32_t* ring_v;
  const int32_t* ring_id;
  long long* ring_ctr;  // [C_N]
};

}  // namespace tr
