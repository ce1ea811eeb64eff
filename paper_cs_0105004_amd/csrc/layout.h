// layout.h -- device-resident state of one scenario slot, shared by the host
// side of libtransims and its kernels.
//
// Vehicles are stored per lane as an ordered queue (lead first) in a ring
// buffer with one record slot per cell of the lane: vehicles never overtake
// inside a lane, so the order only changes when a vehicle enters at the rear
// (parking, arrival from an upstream node, lane change) or leaves at the
// front (next link, trip end) -- or moves sideways.  A record is
//   hot  = { xvf, id }   8 bytes, read and its xvf word rewritten every step
//   cold = { rp, nxt }   8 bytes, read only when the vehicle is near a node
// xvf packs x (bits 0-15), v (bits 16-19) and flags (bits 20-24: last link;
// lowest and highest lane from which the next turn is made).
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

// lane summary written by the front kernel for the back kernel
//   x = target lane id of the lead vehicle (-1: not near the node, -2: trip
//       ends at the node), y = x of the rearmost vehicle (len if empty)

struct DevScen {
  uint32_t flags;
  int32_t vmax;
  uint32_t key0, key1;  // Philox key = seed
  uint64_t slow_thr;
  uint64_t lc_thr;
  int32_t lc_desp;
  int32_t t;  // index of the next step
  int32_t n_links, n_lanes, n_tiles, n_veh;
  int32_t ring_L, ring_n;
  int32_t lc_cells;  // largest lanes*len of a link that changes lanes
  int32_t pad0;
  int64_t n_route;
  // links, in the library's internal (tile) order
  const int32_t* link_len;
  const int8_t* link_lanes;
  const int32_t* link_lane0;  // lane id of lane 0
  const int32_t* link_to;
  const int8_t* link_rank;
  const int32_t* link_ext;    // caller's link id
  const int32_t* node_in_off; // in-links of a node, sorted by rank
  const int32_t* node_in;
  const int32_t* conn_off;
  const int32_t* conn_out;
  const int8_t* conn_lo;
  const int8_t* conn_hi;
  // lanes
  const int32_t* lane_link;
  const int32_t* lane_base;  // first record slot of the lane's ring buffer
  int2* lane_hc;             // {head, count}
  int2* lane_sum;            // see above
  int4* hand_a;              // arrival handoff {tag = t, xvf, id, rp}
  int32_t* hand_nxt;         // arrival handoff: next link
  // vehicle records
  uint2* hot;
  int2* cold;
  // tiles
  const int2* tile_lanes;  // {first lane, lanes}
  long long* tile_ctr;     // [n_tiles * C_N]
  // parking queues per link, ordered by (depart, id)
  const int32_t* wait_off;
  const int32_t* wait_id;
  const int32_t* wait_dep;
  int32_t* wait_head;
  // routes (internal link ids)
  const int64_t* route_off;
  const int32_t* route_links;
  int32_t* exit_t;
  // ring mode (vehicles in cyclic order)
  int32_t* ring_x;
  int32_t* ring_v;
  const int32_t* ring_id;
  long long* ring_ctr;  // [C_N]
  uint32_t* err;
};

}  // namespace tr
