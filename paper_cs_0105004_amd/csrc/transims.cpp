// transims.cpp -- host side of libtransims: input checks, link tiling,
// device layout, launches.  See include/transims.h for the contract.
#include "transims.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "layout.h"
#include "tiler.h"

using namespace tr;

namespace {

constexpr int kDefaultTileLanes = 16;
// scenarios with lane changes: the lane-change sub-step favours fewer,
// larger tiles than the move sub-step alone
constexpr int kDefaultLcTileLanes = 32;
constexpr int kDefaultBackPieces = 4;
constexpr int kDefaultGraphSteps = 64;
// one-kernel steps: a tile also stops at this many cells, so that no
// wavefront is left with a much longer queue of vehicles than the rest
// (on the Portland-sized network at its demand peak 12.8 us per step
// against 13.3 us with 2,048 cells; 12.2 vs 12.6 us over the whole run)
constexpr int kDefaultTileCells = 1024;
// tiles of scenarios with lane changes (their cell cap also bounds the
// lane-change lattice in LDS)
constexpr int kDefaultLcTileCells = 4096;

struct Slot {
  bool net = false, veh = false, ring = false;
  sim_params p{};
  int32_t n_nodes = 0, n_links = 0, n_lanes = 0, n_tiles = 0, n_ftiles = 0, n_veh = 0;
  int64_t n_route = 0, n_records = 0, n_cells = 0;
  std::vector<int32_t> ext_of, int_of;  // internal <-> caller link ids
  std::vector<int32_t> len, lanes, lane0, from, to, base;  // internal order
  std::vector<int4> lane_info;
  std::vector<int32_t> conn_off, conn_out;  // internal ids (turn lanes)
  std::vector<int8_t> conn_lo, conn_hi;
  std::vector<int2> tiles, ftiles;  // move sub-step / lane-change sub-step
  std::vector<int4> plans;  // signal plans {cycle, red, offset mod cycle, 0}
  ExportBufs exp{};         // state export staging in the workspace
  std::vector<double> weight;  // internal order
  std::vector<double> ftile_w;  // summed link weight of each tile
  bool measured = false;        // weights are measured costs (link_cost)
  // each tile's planned load: sum over its links of (routes using the link)
  // x (cells of the link), from the vehicles' plans
  std::vector<double> ftile_plan;
  uint8_t* ws = nullptr;
  uint64_t ws_bytes = 0, ws_net = 0;
  DevScen d{};
  int32_t t = 0;
  int32_t lc_words = 0;
  bool fused = false;  // one kernel per step (state kept by step parity)
  sim_tiling tiling{};
};

}  // namespace

struct sim_ctx {
  sim_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<Slot> slots;
  DevScen* d_descs = nullptr;
  int4* d_work = nullptr;
  long long* d_snap = nullptr;  // per work position, for the tile order
  size_t work_cap = 0;
  int* d_list = nullptr;  // network slots, then ring slots
  size_t list_cap = 0;
  unsigned long long* d_stats = nullptr;
  // the (slot, load generation) pairs the work list was built for; a
  // slot's generation changes with every load and unload, so a work list
  // is never reused for a slot whose contents changed
  std::vector<int64_t> work_key;
  std::vector<uint32_t> slot_gen;
  int n_work = 0, n_net = 0, n_ring = 0, lc_words = 0;
  // the work list holds the tiles of fused slots first (n_fwork items, one
  // kernel per step), then those of two-kernel slots
  int n_fwork = 0;
  int fused_slot = -1;   // the only fused slot of the work list, or -1
  int single_slot = -1;  // the only two-kernel slot of the work list, or -1
  int n_extra = 0;       // extra move wavefronts of the single slot
  // a HIP graph of graph_steps steps of the current work list, and one of
  // the last remainder length (a call of fewer steps, or the steps left
  // after whole replays), reused while calls keep that length
  hipGraphExec_t graph = nullptr;
  int graph_k = 0;
  hipGraphExec_t rgraph = nullptr;
  int rgraph_k = 0;
  // kernel timing
  bool profile = false;
  std::vector<hipEvent_t> events;  // pairs around direct launches
  std::vector<int> event_kind;     // kind of each pair
  size_t n_pairs = 0;
  // profiled graphs: an event before the first kernel and after each one
  hipGraphExec_t pgraph = nullptr;
  int pgraph_k = 0;
  std::vector<hipEvent_t> gev;
  std::vector<int> gkind;  // kernel kind of each interval of a profiled graph
  // the host work plan of the last sim_step_noalloc call, kept until the
  // next one (its upload reads it)
  std::vector<int4> nowork;
  std::vector<int32_t> nolist;
  int64_t acc_launches[4] = {0, 0, 0, 0};
  double acc_ms[4] = {0, 0, 0, 0};
  // last error text of each calling thread (loads may run on other
  // threads than the one that steps)
  std::mutex err_mu;
  std::map<std::thread::id, std::string> err;
};

namespace {

sim_status fail(sim_ctx* c, sim_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) {
    std::lock_guard<std::mutex> lk(c->err_mu);
    c->err[std::this_thread::get_id()] = buf;
  }
  return st;
}

#define HIPCHK(ctx, expr)                                                   \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(ctx, SIM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carve {
  uint8_t* base;
  uint64_t off;
  template <class T>
  T* take(int64_t n) {
    off = (off + 255) & ~uint64_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (uint64_t)std::max<int64_t>(n, 1) * sizeof(T);
    return p;
  }
};

bool lc_link(const sim_params& p, int lanes) {
  return (p.flags & SIM_FLAG_LANE_CHANGE) && lanes >= 2;
}

struct NetDims {
  int64_t L, Q, rec, nodes, conn, xcap;
};

constexpr int64_t kExtraRunsMax = 1024;  // extra move wavefronts per step
constexpr int32_t kMaxGraphSteps = 4096;  // steps per HIP graph
// a remainder of at least this many steps runs as a cached graph of its
// own; shorter ones are launched kernel by kernel
constexpr int32_t kMinRestGraph = 8;

// entries of the list of extra move wavefronts for `tiles` tiles, a
// multiple of 8: the move kernel gives them its first blocks, and the
// tiles after them keep their XCD (block mod 8)
int64_t extra_cap(int64_t tiles, int pieces) {
  const int64_t n = tiles * std::max(pieces - 1, 0);
  return std::min<int64_t>((n + 7) / 8 * 8, kExtraRunsMax);
}

// device arrays of the network part; pointers are null when measuring
void carve_network(Carve& cv, const NetDims& nd, DevScen& d, bool ring) {
  const int64_t L = nd.L, Q = nd.Q;
  d.link_ext = cv.take<int32_t>(L);
  d.lane_info = cv.take<int4>(Q);
  d.lane_state = cv.take<int4>(2 * Q);  // two step-parity buffers
  d.lane_sum = cv.take<int4>(Q);
  d.claim = cv.take<int32_t>(2 * Q);
  d.hand_a = cv.take<int4>(2 * Q);
  d.hand_b = cv.take<int32_t>(2 * Q);
  d.qnext = cv.take<int32_t>(2 * Q);
  d.lane_bm = cv.take<int2>(Q);
  d.tile_live = cv.take<unsigned long long>(2 * Q);  // at most one tile per lane
  d.tile_wake = cv.take<int32_t>(2 * Q);
  d.arr_bits = cv.take<unsigned long long>(2 * ((Q + 63) / 64));
  d.plans = cv.take<int4>(kMaxPlans);
  d.lane_qend = cv.take<int32_t>(Q);
  d.hand_tag = cv.take<int32_t>(2 * Q);
  d.lane_qhead = cv.take<int32_t>(Q);
  d.lane_qrec = cv.take<int4>(Q);
  d.hot = cv.take<uint2>(ring ? 0 : nd.rec);
  d.cold = cv.take<int2>(ring ? 0 : nd.rec);
  d.tile_ctr = cv.take<long long>(Q * C_N);  // at most one tile per lane
  d.ftile_ctr = cv.take<long long>(Q * C_N);
  d.tile_np = cv.take<int32_t>(Q);  // at most one tile per lane
  d.xlist = cv.take<int4>(nd.xcap);
  d.xcount = cv.take<int32_t>(2);
  d.ring_ctr = cv.take<long long>(C_N);
  d.err = cv.take<uint32_t>(1);
}

// vehicle arrays, then the staging area sim_read_state exports the
// per-vehicle state through (15 bytes per vehicle), so that reading a
// state back allocates nothing
void carve_vehicles(Carve& cv, int64_t n, int64_t R, DevScen& d, bool ring,
                    ExportBufs& o) {
  d.wait_rec = cv.take<int4>(ring ? 0 : n);
  d.route_off = cv.take<int64_t>(ring ? 0 : n + 1);
  d.route_info = cv.take<uint32_t>(R);
  d.exit_t = cv.take<int32_t>(R);
  d.ring_x = cv.take<int32_t>(ring ? n : 0);
  d.ring_v = cv.take<int32_t>(ring ? n : 0);
  d.ring_id = cv.take<int32_t>(ring ? n : 0);
  o.status = cv.take<int8_t>(n);
  o.link = cv.take<int32_t>(n);
  o.lane = cv.take<int8_t>(n);
  o.x = cv.take<int32_t>(n);
  o.v = cv.take<int8_t>(n);
  o.rptr = cv.take<int32_t>(n);
}

sim_status check_params(sim_ctx* c, const sim_params* p) {
  if (!p) return fail(c, SIM_E_INVAL, "params is NULL");
  if (p->vmax < 1 || p->vmax > 7) return fail(c, SIM_E_INVAL, "vmax must be 1..7");
  if (p->slow_thr > (1ull << 32) || p->lc_thr > (1ull << 32))
    return fail(c, SIM_E_INVAL, "thresholds must be <= 2^32");
  if (p->lc_desp < 1) return fail(c, SIM_E_INVAL, "lc_desp must be >= 1");
  if (p->flags & ~(SIM_FLAG_RING | SIM_FLAG_LANE_CHANGE | SIM_FLAG_TURN_LANES))
    return fail(c, SIM_E_INVAL, "unknown flag bits");
  return SIM_OK;
}

sim_status check_network(sim_ctx* c, const sim_params* p, const sim_network* n) {
  if (!n) return fail(c, SIM_E_INVAL, "network is NULL");
  const bool ring = p->flags & SIM_FLAG_RING;
  if (n->n_links < 1) return fail(c, SIM_E_INVAL, "need at least one link");
  if (!n->len || !n->lanes || (!ring && (!n->from || !n->to || !n->rank)))
    return fail(c, SIM_E_INVAL, "missing link arrays");
  if (ring) {
    if (n->n_links != 1 || n->lanes[0] != 1)
      return fail(c, SIM_E_INVAL, "ring mode needs one single-lane link");
    if (n->len[0] < 1 || n->len[0] > 32767)
      return fail(c, SIM_E_INVAL, "ring length must be 1..32767");
    return SIM_OK;
  }
  if (n->n_nodes < 1) return fail(c, SIM_E_INVAL, "need nodes");
  std::vector<uint8_t> seen((size_t)n->n_nodes * 128, 0);
  for (int32_t l = 0; l < n->n_links; ++l) {
    if (n->lanes[l] < 1 || n->lanes[l] > 4)
      return fail(c, SIM_E_INVAL, "link %d: lanes must be 1..4", l);
    if (n->len[l] < p->vmax + 1 || n->len[l] > 32767)
      return fail(c, SIM_E_INVAL, "link %d: length must be vmax+1..32767", l);
    if (n->link_cost && !(std::isfinite(n->link_cost[l]) && n->link_cost[l] >= 0.0f))
      return fail(c, SIM_E_INVAL, "link %d: link_cost must be finite and >= 0", l);
    if (n->from[l] < 0 || n->from[l] >= n->n_nodes || n->to[l] < 0 ||
        n->to[l] >= n->n_nodes)
      return fail(c, SIM_E_INVAL, "link %d: node out of range", l);
    if (n->from[l] == n->to[l])
      return fail(c, SIM_E_INVAL, "link %d is a self-loop", l);
    if (n->rank[l] < 0) return fail(c, SIM_E_INVAL, "link %d: negative rank", l);
    uint8_t& f = seen[(size_t)n->to[l] * 128 + (size_t)n->rank[l]];
    if (f)
      return fail(c, SIM_E_INVAL, "two links enter node %d with rank %d",
                  n->to[l], n->rank[l]);
    f = 1;
  }
  if (n->signal_plan) {
    if (n->n_plans < 1 || n->n_plans > kMaxPlans)
      return fail(c, SIM_E_INVAL, "1..%d signal plans", kMaxPlans);
    if (!n->plan_cycle || !n->plan_red || !n->plan_offset)
      return fail(c, SIM_E_INVAL, "signal plan arrays are NULL");
    for (int32_t j = 0; j < n->n_plans; ++j)
      if (n->plan_cycle[j] < 1 || n->plan_red[j] < 0 ||
          n->plan_red[j] > n->plan_cycle[j] || n->plan_offset[j] < 0)
        return fail(c, SIM_E_INVAL, "signal plan %d out of range", j);
    for (int32_t l = 0; l < n->n_links; ++l)
      if (n->signal_plan[l] < -1 || n->signal_plan[l] >= n->n_plans)
        return fail(c, SIM_E_INVAL, "link %d: signal plan out of range", l);
  }
  if (p->flags & SIM_FLAG_TURN_LANES) {
    if (!n->conn_off || !n->conn_out || !n->conn_lo || !n->conn_hi)
      return fail(c, SIM_E_INVAL, "turn lanes need the lane connectivity table");
    if (n->conn_off[0] != 0)
      return fail(c, SIM_E_INVAL, "conn_off[0] must be 0");
    for (int32_t l = 0; l < n->n_links; ++l) {
      if (n->conn_off[l + 1] < n->conn_off[l])
        return fail(c, SIM_E_INVAL, "conn_off must not decrease");
      for (int64_t e = n->conn_off[l]; e < n->conn_off[l + 1]; ++e) {
        const int32_t o = n->conn_out[e];
        if (o < 0 || o >= n->n_links || n->from[o] != n->to[l])
          return fail(c, SIM_E_INVAL, "link %d: bad connectivity entry", l);
        if (n->conn_lo[e] < 0 || n->conn_lo[e] > n->conn_hi[e] ||
            n->conn_hi[e] >= n->lanes[l])
          return fail(c, SIM_E_INVAL, "link %d: bad turn lanes", l);
      }
    }
    if (n->conn_off[n->n_links] > INT32_MAX)
      return fail(c, SIM_E_CAPACITY, "connectivity table too large");
  }
  return SIM_OK;
}

NetDims net_dims(const sim_params* p, const sim_network* n, int pieces) {
  NetDims nd{n->n_links, 0, 0, std::max(n->n_nodes, 1), 0, 0};
  for (int32_t l = 0; l < n->n_links; ++l) {
    nd.Q += n->lanes[l];
    nd.rec += (int64_t)n->lanes[l] * n->len[l] * (lc_link(*p, n->lanes[l]) ? 2 : 1);
  }
  if ((p->flags & SIM_FLAG_TURN_LANES) && n->conn_off) nd.conn = n->conn_off[n->n_links];
  nd.xcap = extra_cap(nd.Q, pieces);  // tiles <= lanes
  return nd;
}

sim_status check_slot(sim_ctx* c, int32_t slot) {
  if (!c) return SIM_E_INVAL;
  if (slot < 0 || slot >= (int32_t)c->slots.size())
    return fail(c, SIM_E_INVAL, "slot %d out of range", slot);
  return SIM_OK;
}

// Route offsets of n vehicles: route_off[0] = 0 and strictly rising (every
// route holds at least one link), so that every route lies inside
// [0, route_off[n]).
sim_status check_route_off(sim_ctx* c, int32_t n, const int64_t* route_off) {
  if (n == 0) return SIM_OK;
  if (!route_off) return fail(c, SIM_E_INVAL, "route_off is NULL");
  if (route_off[0] != 0) return fail(c, SIM_E_INVAL, "route_off[0] must be 0");
  for (int32_t i = 0; i < n; ++i)
    if (route_off[i + 1] <= route_off[i])
      return fail(c, SIM_E_INVAL, "vehicle %d: empty route", i);
  if (route_off[n] > INT32_MAX - 2)
    return fail(c, SIM_E_CAPACITY, "too many route entries");
  return SIM_OK;
}

// With step_mode 2 the one-kernel step skips lanes that are empty and stay
// empty: less memory traffic for one more dependent round of loads per
// tile, which measured no faster on the Portland-sized network (13.9 vs
// 13.3 us per step at its demand peak) nor on 64 batched replications
// (49.3 vs 48.5 us), so the default reads every lane.
bool skip_lanes(const sim_ctx* c, int /*n_fwork*/) {
  return c->cfg.step_mode == 2;
}

// A graph replay first orders the two-kernel work list by the tiles'
// measured times when it holds more tiles than are resident at once (so
// that the order decides when each tile starts) and the ordering kernel
// takes its per-XCD share.  On the 200,000-link network this took the
// whole horizon from 48.2 to 47.2 us per step; on the 64 batched
// replications (one kernel per step) the order the routes plan was as good,
// so the one-kernel list keeps it.
constexpr int kOrderMinTiles = 6144;
bool order_tiles(int n_work) {
  return n_work > kOrderMinTiles && n_work <= 8 * kOrderMax;
}

// Host threads for encoding `work` route entries: one per 2^20 entries, at
// most 16 (the host share of one GPU) and at most the machine's threads.
int host_workers(int64_t work) {
  const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
  return (int)std::max<int64_t>(
      1, std::min<int64_t>({16, hw, work >> 20}));
}

// Calls fn(lo, hi, worker) on `workers` contiguous ranges of [0, n), each
// on a thread of its own (the calling thread takes range 0).
template <class F>
void parallel_ranges(int32_t n, int workers, F&& fn) {
  if (workers <= 1) {
    fn(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(workers - 1);
  auto lo = [&](int w) { return (int32_t)((int64_t)n * w / workers); };
  for (int w = 1; w < workers; ++w)
    th.emplace_back([&, w] { fn(lo(w), lo(w + 1), w); });
  fn(lo(0), lo(1), 0);
  for (std::thread& t : th) t.join();
}

template <class T>
hipError_t up(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

// ---------------------------------------------------------------------------

static sim_status create_body(const sim_config* cfg, sim_ctx** out) {
  if (!cfg || !out) return SIM_E_INVAL;
  *out = nullptr;
  if (cfg->abi_version != SIM_ABI_VERSION) return SIM_E_ABI;
  if (cfg->max_slots < 1 || cfg->max_slots > 65536) return SIM_E_INVAL;
  if (cfg->tile_lanes < 0 || cfg->tile_lanes > kMaxTileLanes) return SIM_E_INVAL;
  if (cfg->back_pieces < 0 || cfg->back_pieces > 8) return SIM_E_INVAL;
  if (cfg->step_mode < 0 || cfg->step_mode > 2) return SIM_E_INVAL;
  if (cfg->graph_steps > kMaxGraphSteps) return SIM_E_INVAL;
  if (cfg->tile_cells != 0 && (cfg->tile_cells < 64 || cfg->tile_cells > 65536))
    return SIM_E_INVAL;
  if (cfg->reserved != 0) return SIM_E_INVAL;
  sim_ctx* c = new (std::nothrow) sim_ctx();
  if (!c) return SIM_E_CAPACITY;
  c->cfg = *cfg;
  if (c->cfg.back_pieces == 0) c->cfg.back_pieces = kDefaultBackPieces;
  if (c->cfg.graph_steps == 0) c->cfg.graph_steps = kDefaultGraphSteps;
  c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  try {
    c->slots.resize(cfg->max_slots);
    c->slot_gen.assign(cfg->max_slots, 0u);
  } catch (const std::bad_alloc&) {
    delete c;
    return SIM_E_CAPACITY;
  }
  if (hipGetDevice(&c->device) != hipSuccess ||
      scratch_init(c->device) != hipSuccess ||
      hipMalloc(&c->d_descs, sizeof(DevScen) * cfg->max_slots) != hipSuccess ||
      hipMalloc(&c->d_stats, sizeof(unsigned long long) * (C_N + 3)) !=
          hipSuccess) {
    sim_destroy(c);
    return SIM_E_DEVICE;
  }
  *out = c;
  return SIM_OK;
}

extern "C" sim_status sim_destroy(sim_ctx* c) {
  if (!c) return SIM_E_INVAL;
  if (c->stream || c->d_descs) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->gev) (void)hipEventDestroy(e);
  if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
  if (c->d_descs) (void)hipFree(c->d_descs);
  if (c->d_stats) (void)hipFree(c->d_stats);
  if (c->d_work) (void)hipFree(c->d_work);
  if (c->d_snap) (void)hipFree(c->d_snap);
  if (c->d_list) (void)hipFree(c->d_list);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->rgraph) (void)hipGraphExecDestroy(c->rgraph);
  delete c;
  return SIM_OK;
}

extern "C" const char* sim_last_error(const sim_ctx* c) {
  if (!c) return "no context";
  sim_ctx* m = const_cast<sim_ctx*>(c);
  std::lock_guard<std::mutex> lk(m->err_mu);
  return m->err[std::this_thread::get_id()].c_str();
}

static sim_status footprint_body(const sim_ctx* cc, const sim_params* p,
                                 const sim_network* net,
                                 const sim_vehicles* veh, uint64_t* bytes) {
  sim_ctx* c = const_cast<sim_ctx*>(cc);
  if (!bytes) return fail(c, SIM_E_INVAL, "bytes is NULL");
  sim_status st = check_params(c, p);
  if (st != SIM_OK) return st;
  if ((st = check_network(c, p, net)) != SIM_OK) return st;
  const bool ring = p->flags & SIM_FLAG_RING;
  DevScen d{};
  Carve cv{nullptr, 0};
  carve_network(cv, net_dims(p, net, c ? c->cfg.back_pieces : kDefaultBackPieces), d, ring);
  if (veh) {
    if (veh->n < 0) return fail(c, SIM_E_INVAL, "negative vehicle count");
    if (!ring && (st = check_route_off(c, veh->n, veh->route_off)) != SIM_OK) return st;
    const int64_t R = (!ring && veh->n > 0) ? veh->route_off[veh->n] : 0;
    ExportBufs o{};
    carve_vehicles(cv, veh->n, R, d, ring, o);
  }
  *bytes = cv.off + 256;
  return SIM_OK;
}

// Loads may run on another host thread than the one that steps: make the
// context's device current on the calling thread.
static sim_status use_device(sim_ctx* c) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    HIPCHK(c, hipSetDevice(c->device));
  return SIM_OK;
}

static sim_status load_network_body(sim_ctx* c, int32_t slot,
                                    const sim_params* p,
                                    const sim_network* net, void* dev_ws,
                                    uint64_t ws_bytes) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  if ((st = use_device(c)) != SIM_OK) return st;
  // from here on the slot holds no scenario, also if the call fails; as in
  // sim_unload, work already enqueued for it finishes first
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Slot& S = c->slots[slot];
  S = Slot();
  ++c->slot_gen[slot];
  if ((st = check_params(c, p)) != SIM_OK) return st;
  if ((st = check_network(c, p, net)) != SIM_OK) return st;
  if (!dev_ws) return fail(c, SIM_E_INVAL, "workspace is NULL");
  S.p = *p;
  S.ring = p->flags & SIM_FLAG_RING;
  const int32_t L = net->n_links;
  S.n_links = L;
  S.n_nodes = S.ring ? 1 : net->n_nodes;

  // ---- tiling: ORB order of links, then whole links packed into tiles
  std::vector<double> w(L);
  for (int32_t l = 0; l < L; ++l)
    w[l] = net->link_cost ? (double)net->link_cost[l]
                          : (double)net->len[l] * net->lanes[l];
  std::vector<int32_t> order(L);
  std::iota(order.begin(), order.end(), 0);
  if (!S.ring && net->node_xy) {
    std::vector<double> mx(L), my(L);
    for (int32_t l = 0; l < L; ++l) {
      mx[l] = 0.5 * (net->node_xy[2 * net->from[l]] + net->node_xy[2 * net->to[l]]);
      my[l] = 0.5 * (net->node_xy[2 * net->from[l] + 1] +
                     net->node_xy[2 * net->to[l] + 1]);
    }
    orb_order(order, mx, my, w);
  }
  S.ext_of = order;
  S.int_of.assign(L, 0);
  for (int32_t i = 0; i < L; ++i) S.int_of[order[i]] = i;
  S.len.resize(L);
  S.lanes.resize(L);
  S.lane0.resize(L);
  S.from.resize(L);
  S.to.resize(L);
  S.weight.resize(L);
  int32_t q = 0;
  for (int32_t i = 0; i < L; ++i) {
    const int32_t e = order[i];
    S.len[i] = net->len[e];
    S.lanes[i] = net->lanes[e];
    S.lane0[i] = q;
    S.from[i] = S.ring ? 0 : net->from[e];
    S.to[i] = S.ring ? 0 : net->to[e];
    S.weight[i] = w[e];
    q += S.lanes[i];
    S.n_cells += (int64_t)S.len[i] * S.lanes[i];
  }
  S.n_lanes = q;
  {
    int32_t min_len = INT32_MAX;
    for (int32_t i = 0; i < L; ++i) min_len = std::min(min_len, S.len[i]);
    S.fused = !S.ring && c->cfg.step_mode != 1 &&
              !(p->flags & SIM_FLAG_LANE_CHANGE) && min_len >= 2 * p->vmax;
  }
  // one-kernel tiles and tiles of lane-changing links are capped in cells
  // (the latter bound the lane-change lattice in LDS)
  const bool lc_slot = !S.ring && (p->flags & SIM_FLAG_LANE_CHANGE);
  const int tile_lanes = c->cfg.tile_lanes != 0 ? c->cfg.tile_lanes
                         : lc_slot              ? kDefaultLcTileLanes
                                                : kDefaultTileLanes;
  const int tile_cells = c->cfg.tile_cells != 0 ? c->cfg.tile_cells
                         : lc_slot              ? kDefaultLcTileCells
                                                : kDefaultTileCells;
  S.ftiles = (S.fused || lc_slot)
                 ? pack_tiles(S.lanes, S.len, tile_lanes, tile_cells)
                 : pack_tiles(S.lanes, tile_lanes);
  if (net->link_cost && !S.ring) {
    // adaptive load balancing: with measured per-link costs the cost takes
    // over from the cell count as what cuts the tiles.  The cell cap is
    // doubled, and a tile also stops at the mean measured cost of the tiles
    // the lane cap and that doubled cell cap alone would make, so that the
    // links that cost most get tiles of their own while the costliest
    // tiles shrink and the cheap ones grow.
    const int64_t cells = (S.fused || lc_slot)
                              ? std::min<int64_t>(2 * (int64_t)tile_cells, 65536)
                              : INT64_MAX;
    const size_t n_base =
        (S.fused || lc_slot) ? pack_tiles(S.lanes, S.len, tile_lanes, (int)cells).size()
                             : S.ftiles.size();
    double total = 0.0;
    for (int32_t i = 0; i < L; ++i) total += S.weight[i];
    const double cap = total / (double)std::max<size_t>(n_base, 1);
    if (cap > 0.0)
      S.ftiles = pack_tiles(S.lanes, S.len, S.weight, tile_lanes, cells, cap);
  }
  S.n_ftiles = (int32_t)S.ftiles.size();
  S.ftile_plan.clear();  // set again when vehicles are loaded
  S.measured = net->link_cost != nullptr && !S.ring;
  S.ftile_w.assign(S.ftiles.size(), 0.0);
  {
    int32_t l = 0;
    for (size_t t = 0; t < S.ftiles.size(); ++t)
      for (; l < L && S.lane0[l] < S.ftiles[t].x + S.ftiles[t].y; ++l)
        S.ftile_w[t] += S.weight[l];
  }
  S.lc_words = 0;
  if (lc_slot) {
    int32_t l = 0;
    for (const int2& tl : S.ftiles) {
      int32_t words = 0;
      for (; l < L && S.lane0[l] < tl.x + tl.y; ++l)
        if (lc_link(*p, S.lanes[l])) words += S.lanes[l] * ((S.len[l] + 31) / 32);
      S.lc_words = std::max(S.lc_words, words);
    }
    if (S.lc_words > kMaxLcWords)
      return fail(c, SIM_E_CAPACITY, "lane-change lattice of %d words", S.lc_words);
  }
  S.tiles = S.ftiles;  // the move sub-step splits these tiles further
  S.n_tiles = S.n_ftiles;
  S.tiling = tiling_metrics(S.tiles, S.lanes, S.lane0, S.weight);
  S.tiling.n_lanes = S.n_lanes;
  S.tiling.n_cells = S.n_cells;

  // ---- host images of the device arrays
  NetDims nd = net_dims(p, net, c->cfg.back_pieces);
  if (S.n_lanes >= (1 << 24))
    return fail(c, SIM_E_CAPACITY, "at most %d lanes per scenario", (1 << 24) - 1);
  S.conn_off.assign(L + 1, 0);
  if (p->flags & SIM_FLAG_TURN_LANES) {
    for (int32_t i = 0; i < L; ++i) {
      const int32_t e = order[i];
      for (int64_t k = net->conn_off[e]; k < net->conn_off[e + 1]; ++k) {
        S.conn_out.push_back(S.int_of[net->conn_out[k]]);
        S.conn_lo.push_back(net->conn_lo[k]);
        S.conn_hi.push_back(net->conn_hi[k]);
      }
      S.conn_off[i + 1] = (int32_t)S.conn_out.size();
    }
  }
  std::vector<int4>& lane_info = S.lane_info;
  lane_info.assign(S.n_lanes, make_int4(0, 0, 0, 0));
  S.base.resize(L);
  int64_t rec = 0;
  for (int32_t i = 0; i < L; ++i) {
    const int cap = S.len[i] * (lc_link(*p, S.lanes[i]) ? 2 : 1);
    S.base[i] = (int32_t)rec;
    const int rank = S.ring ? 0 : net->rank[order[i]];
    for (int k = 0; k < S.lanes[i]; ++k) {
      lane_info[S.lane0[i] + k] =
          make_int4((int32_t)rec,
                    (int32_t)lmeta_make(S.len[i], k, S.lanes[i], rank,
                                        (!S.ring && net->signal_plan)
                                            ? net->signal_plan[order[i]] : -1),
                    i, 0);
      rec += cap;
    }
    if (rec > INT32_MAX) return fail(c, SIM_E_CAPACITY, "too many cells");
  }
  S.n_records = rec;

  // ---- carve and upload
  DevScen& d = S.d;
  Carve cv{static_cast<uint8_t*>(dev_ws), 0};
  carve_network(cv, nd, d, S.ring);
  if (cv.off > ws_bytes)
    return fail(c, SIM_E_NOMEM, "workspace of %llu bytes, network needs %llu",
                (unsigned long long)ws_bytes, (unsigned long long)cv.off);
  S.ws = static_cast<uint8_t*>(dev_ws);
  S.ws_bytes = ws_bytes;
  S.ws_net = cv.off;
  d.flags = p->flags;
  d.vmax = p->vmax;
  d.key0 = (uint32_t)p->seed;
  d.key1 = (uint32_t)(p->seed >> 32);
  d.slow_thr = p->slow_thr;
  d.lc_thr = p->lc_thr;
  d.lc_desp = p->lc_desp;
  d.n_links = L;
  d.n_lanes = S.n_lanes;
  d.n_tiles = S.n_tiles;
  d.n_ftiles = S.n_ftiles;
  d.xcap = (S.ring || S.fused) ? 0 : (int32_t)extra_cap(S.n_ftiles, c->cfg.back_pieces);
  d.n_plans = (!S.ring && net->signal_plan) ? net->n_plans : 0;
  d.fused = S.fused ? 1 : 0;
  d.lc_words = S.lc_words;
  d.ring_L = S.ring ? net->len[0] : 0;
  hipStream_t s = c->stream;
  HIPCHK(c, up(const_cast<int32_t*>(d.link_ext), S.ext_of.data(), L, s));
  HIPCHK(c, up(const_cast<int4*>(d.lane_info), lane_info.data(), S.n_lanes, s));
  if (d.n_plans > 0) {
    std::vector<int4>& plans = S.plans;
    plans.resize(d.n_plans);
    for (int32_t j = 0; j < d.n_plans; ++j)
      plans[j] = make_int4(net->plan_cycle[j], net->plan_red[j],
                           net->plan_offset[j] % net->plan_cycle[j], 0);
    HIPCHK(c, up(const_cast<int4*>(d.plans), plans.data(), d.n_plans, s));
  }
  {
    std::vector<int2> bm(S.n_lanes);
    for (int32_t qq = 0; qq < S.n_lanes; ++qq)
      bm[qq] = make_int2(lane_info[qq].x, lane_info[qq].y);
    HIPCHK(c, up(const_cast<int2*>(d.lane_bm), bm.data(), S.n_lanes, s));
  }
  HIPCHK(c, hipStreamSynchronize(s));
  S.net = true;
  ++c->slot_gen[slot];  // slot contents changed: rebuild work lists
  return SIM_OK;
}

static sim_status load_vehicles_body(sim_ctx* c, int32_t slot,
                                     const sim_vehicles* v) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  if ((st = use_device(c)) != SIM_OK) return st;
  Slot& S = c->slots[slot];
  if (!S.net) return fail(c, SIM_E_STATE, "slot %d has no network", slot);
  if (!v || v->n < 0) return fail(c, SIM_E_INVAL, "bad vehicles");
  // the per-run device state is reset below: until this load succeeds the
  // slot holds no vehicles and cannot be stepped
  S.veh = false;
  ++c->slot_gen[slot];
  const int32_t n = v->n;
  const int vmax = S.p.vmax;
  if (n > 0 && !v->depart) return fail(c, SIM_E_INVAL, "depart is NULL");
  if (v->t0 < 0) return fail(c, SIM_E_INVAL, "t0 must be >= 0");
  const bool has_init = v->init_status != nullptr;
  if (has_init && (!v->init_lane || !v->init_x || !v->init_v ||
                   (!S.ring && !v->init_rptr)))
    return fail(c, SIM_E_INVAL, "incomplete initial state arrays");
  if (!S.ring && (st = check_route_off(c, n, v->route_off)) != SIM_OK) return st;
  if (!S.ring && n > 0 && !v->route_links) return fail(c, SIM_E_INVAL, "route_links is NULL");
  DevScen& d = S.d;
  hipStream_t s = c->stream;
  // per-run device state starts empty
  {
    std::vector<int4> hand_a(2 * S.n_lanes, make_int4(kTagNone, 0, 0, 0));
    HIPCHK(c, up(d.hand_a, hand_a.data(), 2 * S.n_lanes, s));
    HIPCHK(c, hipMemsetAsync(d.lane_state, 0, sizeof(int4) * 2 * S.n_lanes, s));
    std::vector<int32_t> tags(2 * S.n_lanes, kTagNone);
    HIPCHK(c, up(d.hand_tag, tags.data(), 2 * S.n_lanes, s));
    HIPCHK(c, hipMemsetAsync(d.tile_ctr, 0, sizeof(long long) * C_N * S.n_lanes, s));
    HIPCHK(c, hipMemsetAsync(d.ftile_ctr, 0, sizeof(long long) * C_N * S.n_ftiles, s));
    HIPCHK(c, hipMemsetAsync(d.xcount, 0, sizeof(int32_t) * 2, s));
    HIPCHK(c, hipMemsetAsync(d.tile_np, 0, sizeof(int32_t) * S.n_lanes, s));
    HIPCHK(c, hipMemsetAsync(d.ring_ctr, 0, sizeof(long long) * C_N, s));
    HIPCHK(c, hipMemsetAsync(d.err, 0, sizeof(uint32_t), s));
    // the one-kernel step starts by looking at every lane of every tile
    std::vector<unsigned long long> live(2 * (size_t)S.n_ftiles, ~0ull);
    HIPCHK(c, up(d.tile_live, live.data(), 2 * (int64_t)S.n_ftiles, s));
    std::vector<int32_t> wake(2 * (size_t)S.n_ftiles, v->t0);
    HIPCHK(c, up(d.tile_wake, wake.data(), 2 * (int64_t)S.n_ftiles, s));
    HIPCHK(c, hipMemsetAsync(d.arr_bits, 0,
                             sizeof(unsigned long long) * 2 * ((S.n_lanes + 63) / 64), s));
    std::vector<int32_t> none(2 * S.n_lanes, INT32_MAX);
    HIPCHK(c, up(d.claim, none.data(), 2 * S.n_lanes, s));
    HIPCHK(c, up(d.qnext, none.data(), 2 * S.n_lanes, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }

  if (S.ring) {
    const int32_t Lr = d.ring_L;
    if (!has_init) return fail(c, SIM_E_INVAL, "ring mode needs initial placement");
    if (n > kRingMax)
      return fail(c, SIM_E_CAPACITY, "ring mode supports up to %d vehicles", kRingMax);
    std::vector<int32_t> idx(n);
    std::vector<uint8_t> used(Lr, 0);
    for (int32_t i = 0; i < n; ++i) {
      if (v->init_status[i] != 1)
        return fail(c, SIM_E_INVAL, "ring mode: vehicle %d must start on the ring", i);
      if (v->init_lane[i] != 0 || v->init_x[i] < 0 || v->init_x[i] >= Lr ||
          v->init_v[i] < 0 || v->init_v[i] > vmax)
        return fail(c, SIM_E_INVAL, "vehicle %d: placement out of range", i);
      if (used[v->init_x[i]]++)
        return fail(c, SIM_E_INVAL, "two vehicles share cell %d", v->init_x[i]);
      idx[i] = i;
    }
    std::sort(idx.begin(), idx.end(),
              [&](int32_t a, int32_t b) { return v->init_x[a] < v->init_x[b]; });
    std::vector<int32_t> rx(n), rv(n), rid(n);
    for (int32_t j = 0; j < n; ++j) {
      rx[j] = v->init_x[idx[j]];
      rv[j] = v->init_v[idx[j]];
      rid[j] = idx[j];
    }
    Carve cv{S.ws, S.ws_net};
    carve_vehicles(cv, n, 0, d, true, S.exp);
    if (cv.off > S.ws_bytes)
      return fail(c, SIM_E_NOMEM, "workspace of %llu bytes, scenario needs %llu",
                  (unsigned long long)S.ws_bytes, (unsigned long long)cv.off);
    d.n_veh = n;
    d.ring_n = n;
    d.t = v->t0;
    HIPCHK(c, up(d.ring_x, rx.data(), n, s));
    HIPCHK(c, up(d.ring_v, rv.data(), n, s));
    HIPCHK(c, up(const_cast<int32_t*>(d.ring_id), rid.data(), n, s));
    S.n_route = 0;
    d.n_route = 0;
  } else {
    const int64_t R = n > 0 ? v->route_off[n] : 0;  // offsets checked above
    const int32_t L = S.n_links;
    const bool turn = S.p.flags & SIM_FLAG_TURN_LANES;
    // route entries as internal link ids, then as route info words; the
    // vehicles are split into contiguous ranges encoded by parallel host
    // threads (tens of millions of entries for the largest scenarios).  The
    // error reported is that of the lowest vehicle index, as a serial pass
    // would report it.
    // (rinfo is filled by the threads without being cleared first, so that
    // its pages are first touched in parallel)
    std::unique_ptr<uint32_t[]> rinfo(new uint32_t[std::max<int64_t>(R, 1)]);
    auto int_link = [&](int64_t j) { return S.int_of[v->route_links[j]]; };
    const int n_workers = host_workers(R);
    std::vector<int32_t> bad_veh(n_workers, INT32_MAX);
    std::vector<const char*> bad_msg(n_workers, nullptr);
    std::vector<std::vector<int32_t>> uses(n_workers);
    parallel_ranges(n, n_workers, [&](int32_t i0, int32_t i1, int wk) {
      std::vector<int32_t>& use = uses[wk];
      use.assign(L, 0);
      for (int32_t i = i0; i < i1; ++i) {
        const int64_t a = v->route_off[i], b = v->route_off[i + 1];
        int32_t prev = -1;
        for (int64_t j = a; j < b; ++j) {
          const int32_t e = v->route_links[j];
          if (e < 0 || e >= L) {
            bad_veh[wk] = i;
            bad_msg[wk] = "route link out of range";
            return;
          }
          const int32_t link = S.int_of[e];
          if (j > a && S.to[prev] != S.from[link]) {
            bad_veh[wk] = i;
            bad_msg[wk] = "route links not connected";
            return;
          }
          ++use[link];
          prev = link;
        }
        for (int64_t j = a; j < b; ++j) {
          const int32_t link = int_link(j);
          int lo = 0, hi = S.lanes[link] - 1;
          if (turn && j + 1 < b) {
            const int32_t next = int_link(j + 1);
            bool found = false;
            for (int32_t e = S.conn_off[link]; e < S.conn_off[link + 1]; ++e)
              if (S.conn_out[e] == next) {
                lo = S.conn_lo[e];
                hi = S.conn_hi[e];
                found = true;
                break;
              }
            if (!found) {
              bad_veh[wk] = i;
              bad_msg[wk] = "no lane connectivity for a turn";
              return;
            }
          }
          rinfo[j] = rinfo_make(S.lane0[link], S.lanes[link], lo, hi, j + 1 == b);
        }
      }
    });
    {
      int wbad = -1;
      for (int wk = 0; wk < n_workers; ++wk)
        if (bad_veh[wk] != INT32_MAX && (wbad < 0 || bad_veh[wk] < bad_veh[wbad]))
          wbad = wk;
      if (wbad >= 0)
        return fail(c, SIM_E_INVAL, "vehicle %d: %s", bad_veh[wbad], bad_msg[wbad]);
    }
    auto ninfo_of = [&](int64_t r, int32_t i) -> int32_t {
      return r + 1 < v->route_off[i + 1] ? (int32_t)rinfo[r + 1] : 0;
    };
    // planned load of each tile (orders the tiles of a launch when no
    // measured costs are given)
    {
      std::vector<double> use(L, 0.0);
      for (const std::vector<int32_t>& u : uses)
        for (int32_t l = 0; l < L; ++l) use[l] += (double)u[l];
      S.ftile_plan.assign(S.ftiles.size(), 0.0);
      int32_t l = 0;
      for (size_t t = 0; t < S.ftiles.size(); ++t)
        for (; l < L && S.lane0[l] < S.ftiles[t].x + S.ftiles[t].y; ++l)
          S.ftile_plan[t] += use[l] * (double)S.len[l];
    }
    // initial state: active vehicles into their lanes, lead first
    std::vector<int32_t> wait_cnt(L + 1, 0);
    std::vector<int32_t> act;
    for (int32_t i = 0; i < n; ++i) {
      const int stt = has_init ? v->init_status[i] : 0;
      if (stt == 0) {
        wait_cnt[int_link(v->route_off[i]) + 1]++;
      } else if (stt == 1) {
        const int32_t rp = v->init_rptr[i];
        if (rp < 0 || v->route_off[i] + rp >= v->route_off[i + 1])
          return fail(c, SIM_E_INVAL, "vehicle %d: rptr out of range", i);
        const int32_t link = int_link(v->route_off[i] + rp);
        const int k = v->init_lane[i];
        if (k < 0 || k >= S.lanes[link] || v->init_x[i] < 0 ||
            v->init_x[i] >= S.len[link] || v->init_v[i] < 0 || v->init_v[i] > vmax)
          return fail(c, SIM_E_INVAL, "vehicle %d: placement out of range", i);
        act.push_back(i);
      } else if (stt != 2) {
        return fail(c, SIM_E_INVAL, "vehicle %d: bad status", i);
      }
    }
    auto link_of = [&](int32_t i) { return int_link(v->route_off[i] + v->init_rptr[i]); };
    auto lane_of = [&](int32_t i) { return S.lane0[link_of(i)] + v->init_lane[i]; };
    std::sort(act.begin(), act.end(), [&](int32_t a, int32_t b) {
      const int32_t qa = lane_of(a), qb = lane_of(b);
      if (qa != qb) return qa < qb;
      return v->init_x[a] > v->init_x[b];
    });
    std::vector<int4> state(S.n_lanes, make_int4(0, 0, 0, 0));
    // records of each lane's run are contiguous from the lane's base
    std::vector<uint2> hot;
    std::vector<int2> cold;
    std::vector<int64_t> run_slot;
    std::vector<int32_t> run_len, run_first;
    for (size_t a = 0; a < act.size();) {
      const int32_t qq = lane_of(act[a]);
      size_t b = a;
      while (b < act.size() && lane_of(act[b]) == qq) ++b;
      const int32_t link = link_of(act[a]);
      run_slot.push_back(S.base[link] + (int64_t)(qq - S.lane0[link]) *
                                            (S.len[link] * (lc_link(S.p, S.lanes[link]) ? 2 : 1)));
      run_len.push_back((int32_t)(b - a));
      run_first.push_back((int32_t)hot.size());
      for (size_t j = a; j < b; ++j) {
        const int32_t i = act[j];
        if (j > a && v->init_x[act[j - 1]] == v->init_x[i])
          return fail(c, SIM_E_INVAL, "vehicles %d and %d share a cell", act[j - 1], i);
        const int64_t rp = v->route_off[i] + v->init_rptr[i];
        hot.push_back(make_uint2(pack_xvf(v->init_x[i], v->init_v[i], rinfo_flags(rinfo[rp])),
                                 (uint32_t)i));
        cold.push_back(make_int2((int32_t)rp, ninfo_of(rp, i)));
      }
      state[qq] = make_int4((int)hot[run_first.back()].x, cold[run_first.back()].y,
                            (int)hot.back().x, hc_make(0, 0, (int)(b - a)));
      a = b;
    }
    // parking queues ordered by (depart, id)
    for (int32_t l = 0; l < L; ++l) wait_cnt[l + 1] += wait_cnt[l];
    std::vector<int32_t> wid(wait_cnt[L]);
    {
      std::vector<int32_t> fill(wait_cnt.begin(), wait_cnt.end() - 1);
      for (int32_t i = 0; i < n; ++i)
        if ((has_init ? v->init_status[i] : 0) == 0) wid[fill[int_link(v->route_off[i])]++] = i;
      for (int32_t l = 0; l < L; ++l)
        std::sort(wid.begin() + wait_cnt[l], wid.begin() + wait_cnt[l + 1],
                  [&](int32_t a, int32_t b) {
                    if (v->depart[a] != v->depart[b]) return v->depart[a] < v->depart[b];
                    return a < b;
                  });
    }
    std::vector<int4> wrec(wid.size());
    for (size_t j = 0; j < wid.size(); ++j) {
      const int32_t i = wid[j];
      const int64_t r0 = v->route_off[i];
      if (v->depart[i] < 0 || v->depart[i] >= (1 << kDepartBits))
        return fail(c, SIM_E_INVAL, "vehicle %d: depart must be 0..2^%d-1", i, kDepartBits);
      wrec[j] = make_int4(i, v->depart[i] | (int)(rinfo_flags(rinfo[r0]) << kDepartBits),
                          (int32_t)r0, ninfo_of(r0, i));
    }
    // each link's queue is kept with its lane 0: head index and head record;
    // every lane of the link knows where the queue ends
    std::vector<int32_t> qhead(S.n_lanes, 0);
    std::vector<int4> qrec(S.n_lanes, make_int4(-1, 0, 0, 0));
    for (int32_t l = 0; l < L; ++l) {
      const int32_t q0 = S.lane0[l];
      qhead[q0] = wait_cnt[l];
      if (wait_cnt[l] < wait_cnt[l + 1]) qrec[q0] = wrec[wait_cnt[l]];
      for (int k = 0; k < S.lanes[l]; ++k) S.lane_info[q0 + k].w = wait_cnt[l + 1];
    }

    Carve cv{S.ws, S.ws_net};
    carve_vehicles(cv, n, R, d, false, S.exp);
    if (cv.off > S.ws_bytes)
      return fail(c, SIM_E_NOMEM, "workspace of %llu bytes, scenario needs %llu",
                  (unsigned long long)S.ws_bytes, (unsigned long long)cv.off);
    d.n_veh = n;
    d.n_route = R;
    d.t = v->t0;
    HIPCHK(c, up(const_cast<int4*>(d.wait_rec), wrec.data(), (int64_t)wrec.size(), s));
    HIPCHK(c, up(d.lane_qhead, qhead.data(), S.n_lanes, s));
    HIPCHK(c, up(d.lane_qrec, qrec.data(), S.n_lanes, s));
    HIPCHK(c, up(const_cast<int4*>(d.lane_info), S.lane_info.data(), S.n_lanes, s));
    {
      std::vector<int32_t> qend(S.n_lanes);
      for (int32_t qq = 0; qq < S.n_lanes; ++qq) qend[qq] = S.lane_info[qq].w;
      HIPCHK(c, up(const_cast<int32_t*>(d.lane_qend), qend.data(), S.n_lanes, s));
    }
    HIPCHK(c, up(const_cast<int64_t*>(d.route_off), v->route_off, n + 1, s));
    HIPCHK(c, up(const_cast<uint32_t*>(d.route_info), rinfo.get(), R, s));
    if (v->exit_t0) {
      HIPCHK(c, up(d.exit_t, v->exit_t0, R, s));
    } else if (R > 0) {  // every entry -1: all bytes 0xFF
      HIPCHK(c, hipMemsetAsync(d.exit_t, 0xFF, sizeof(int32_t) * (size_t)R, s));
    }
    for (size_t r = 0; r < run_slot.size(); ++r) {
      HIPCHK(c, up(d.hot + run_slot[r], hot.data() + run_first[r], run_len[r], s));
      HIPCHK(c, up(d.cold + run_slot[r], cold.data() + run_first[r], run_len[r], s));
    }
    // a fused slot keeps the state of step t in buffer t & 1, with the
    // claims of the lead vehicles near a node registered for that step
    const int64_t cur = S.fused ? (int64_t)(v->t0 & 1) * S.n_lanes : 0;
    HIPCHK(c, up(d.lane_state + cur, state.data(), S.n_lanes, s));
    std::vector<int32_t> qn, cl;
    if (S.fused) {
      qn.assign(S.n_lanes, INT32_MAX);
      for (int32_t l = 0; l < L; ++l)
        if (wait_cnt[l] < wait_cnt[l + 1]) qn[S.lane0[l]] = v->depart[wid[wait_cnt[l]]];
      cl.assign(S.n_lanes, INT32_MAX);
      for (int32_t qq = 0; qq < S.n_lanes; ++qq) {
        if (hc_cnt(state[qq].w) == 0) continue;
        const uint32_t meta = (uint32_t)S.lane_info[qq].y;
        const uint32_t xvf = (uint32_t)state[qq].x, ni = (uint32_t)state[qq].y;
        if (lmeta_len(meta) - 1 - xvf_x(xvf) >= vmax || (xvf_fl(xvf) & kFlLast)) continue;
        // a lead vehicle held by a red light claims nothing in step t0,
        // as in the kernel that registers the claims of later steps
        const int pl = lmeta_plan(meta);
        if (pl >= 0) {
          const int4 q = S.plans[pl];
          if ((int)(((uint32_t)v->t0 + (uint32_t)q.z) % (uint32_t)q.x) < q.y) continue;
        }
        const int k = lmeta_k(meta);
        const int32_t tgt = rinfo_lane0(ni) + std::min(k, rinfo_lanes(ni) - 1);
        cl[tgt] = std::min(cl[tgt], lmeta_rank(meta) * 8 + k);
      }
      HIPCHK(c, up(d.qnext + cur, qn.data(), S.n_lanes, s));
      HIPCHK(c, up(d.claim + cur, cl.data(), S.n_lanes, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    S.n_route = R;
  }
  S.n_veh = n;
  S.t = v->t0;
  d.n_veh = n;
  HIPCHK(c, hipMemcpyAsync(c->d_descs + slot, &d, sizeof(DevScen), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  S.veh = true;
  ++c->slot_gen[slot];
  return SIM_OK;
}

namespace {

// The work list of one set of slots, computed on the host: all tiles of
// all network slots, dealt to the 8 XCDs in contiguous chunks (workgroup w
// runs on XCD w mod 8), fused slots' tiles first (they run in their own
// kernel), then the tiles of two-kernel slots; and the slot list (network
// slots, then ring slots).
struct WorkPlan {
  std::vector<int4> work;
  std::vector<int32_t> list;
  int n_fwork = 0, fused_slot = -1, single_slot = -1, n_extra = 0;
  int lc_words = 0, n_net = 0, n_ring = 0;
};

void plan_work(const sim_ctx* c, const std::vector<int32_t>& net,
               const std::vector<int32_t>& ring, WorkPlan& wp) {
  int lc = 0;
  std::vector<int4>& work = wp.work;
  work.clear();
  std::vector<int32_t> fused_slots, two_slots;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int2> all;
    for (int32_t sl : net) {
      const Slot& S = c->slots[sl];
      if (S.fused != (pass == 0)) continue;
      (pass == 0 ? fused_slots : two_slots).push_back(sl);
      for (int32_t t = 0; t < S.n_ftiles; ++t) all.push_back(make_int2(sl, t));
      if (pass == 1) lc = std::max(lc, S.lc_words);
    }
    std::vector<int2> dealt = xcd_interleave(all, 8);
    // each XCD starts its costliest tiles first (its set of tiles, and so
    // its L2 region, stays the same), which shortens the tail of the
    // launch; the cost is the load the routes plan (routes using a link x
    // its cells), else the measured one.  The planned load orders better
    // than measured cycles: on the Portland-sized and 200k-link networks
    // with cost-capped tiles, 11.82 vs 11.88 and 60.4 vs 63.0 us per step
    bool measured = !all.empty(), planned = !all.empty();
    for (const int2& a : all) {
      measured = measured && c->slots[a.x].measured;
      planned = planned && c->slots[a.x].ftile_plan.size() ==
                               c->slots[a.x].ftiles.size();
    }
    if (measured || planned) {
      auto cost = [&](int2 a) {
        const Slot& S = c->slots[a.x];
        return planned ? S.ftile_plan[a.y] : S.ftile_w[a.y];
      };
      for (size_t x = 0; x < 8; ++x) {
        std::vector<int2> mine;
        for (size_t k = x; k < dealt.size(); k += 8) mine.push_back(dealt[k]);
        std::stable_sort(mine.begin(), mine.end(),
                         [&](int2 a, int2 b) { return cost(a) > cost(b); });
        for (size_t k = x, j = 0; k < dealt.size(); k += 8, ++j) dealt[k] = mine[j];
      }
    }
    for (size_t k = 0; k < dealt.size(); ++k) {
      const int2 tl = c->slots[dealt[k].x].ftiles[dealt[k].y];
      work.push_back(make_int4(dealt[k].x, tl.x, tl.y, dealt[k].y));
    }
    if (pass == 0) wp.n_fwork = (int)work.size();
  }
  wp.fused_slot = fused_slots.size() == 1 ? fused_slots[0] : -1;
  wp.single_slot = two_slots.size() == 1 ? two_slots[0] : -1;
  wp.n_extra = wp.single_slot >= 0 ? c->slots[wp.single_slot].d.xcap : 0;
  wp.list = net;
  wp.list.insert(wp.list.end(), ring.begin(), ring.end());
  wp.lc_words = lc;
  wp.n_net = (int)net.size();
  wp.n_ring = (int)ring.size();
}

sim_status build_work(sim_ctx* c, const std::vector<int32_t>& net,
                      const std::vector<int32_t>& ring) {
  std::vector<int64_t> key;
  for (int32_t sl : net) key.push_back((int64_t)sl << 32 | c->slot_gen[sl]);
  key.push_back(-1);
  for (int32_t sl : ring) key.push_back((int64_t)sl << 32 | c->slot_gen[sl]);
  if (key == c->work_key) return SIM_OK;
  WorkPlan wp;
  plan_work(c, net, ring, wp);
  c->n_fwork = wp.n_fwork;
  c->fused_slot = wp.fused_slot;
  c->single_slot = wp.single_slot;
  c->n_extra = wp.n_extra;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_k = 0;
  }
  if (c->rgraph) {
    (void)hipGraphExecDestroy(c->rgraph);
    c->rgraph = nullptr;
    c->rgraph_k = 0;
  }
  if (c->pgraph) {
    (void)hipGraphExecDestroy(c->pgraph);
    c->pgraph = nullptr;
    c->pgraph_k = 0;
  }
  const std::vector<int4>& work = wp.work;
  const std::vector<int32_t>& list = wp.list;
  // (the lists grow by half again when they must, so that slots coming
  // and going seldom reallocate them)
  if (work.size() > c->work_cap) {
    if (c->d_work) HIPCHK(c, hipFree(c->d_work));
    if (c->d_snap) HIPCHK(c, hipFree(c->d_snap));
    c->d_work = nullptr;
    c->d_snap = nullptr;
    const size_t cap = std::max(work.size(), c->work_cap + c->work_cap / 2);
    HIPCHK(c, hipMalloc(&c->d_work, sizeof(int4) * std::max<size_t>(cap, 1)));
    HIPCHK(c, hipMalloc(&c->d_snap,
                        sizeof(long long) * std::max<size_t>(cap, 1)));
    c->work_cap = cap;
  }
  if (list.size() > c->list_cap) {
    if (c->d_list) HIPCHK(c, hipFree(c->d_list));
    c->d_list = nullptr;
    const size_t cap = std::max(list.size(), c->list_cap + c->list_cap / 2);
    HIPCHK(c, hipMalloc(&c->d_list, sizeof(int) * std::max<size_t>(cap, 1)));
    c->list_cap = cap;
  }
  HIPCHK(c, up(c->d_work, work.data(), (int64_t)work.size(), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_snap, 0, sizeof(long long) * work.size(),
                           c->stream));
  HIPCHK(c, up(c->d_list, list.data(), (int64_t)list.size(), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->n_work = (int)work.size();
  c->n_net = wp.n_net;
  c->n_ring = wp.n_ring;
  c->lc_words = wp.lc_words;
  c->work_key = key;
  return SIM_OK;
}

// A HIP graph of K steps of the current work list (two kernels per step) and
// the advance of t by K, built node by node (the caller's stream may be the
// legacy default stream, which cannot be captured).  A profiled graph also
// records kLeadEvents events back to back, the last of them just before the
// first kernel, and one event after every kernel, so that consecutive events
// bracket one kernel each with no host gap in between.
constexpr int kLeadEvents = 8;  // back-to-back events that time an event

sim_status build_graph(sim_ctx* c, int K, bool profiled, hipGraphExec_t* out) {
  const int n_fw = c->n_fwork, n_tw = c->n_work - c->n_fwork;
  const int per_step = (n_fw > 0 ? 1 : 0) + (n_tw > 0 ? 2 : 0);
  if (profiled) {
    while (c->gev.size() < (size_t)(per_step * K + kLeadEvents)) {
      hipEvent_t ev;
      HIPCHK(c, hipEventCreate(&ev));
      c->gev.push_back(ev);
    }
    c->gkind.clear();
  }
  hipGraph_t g = nullptr;
  HIPCHK(c, hipGraphCreate(&g, 0));
  // one-kernel slots
  const bool fbatched = c->fused_slot < 0;
  int fslot = fbatched ? 0 : c->fused_slot;
  const int4* fwork = c->d_work;
  // two-kernel slots
  const bool batched = c->single_slot < 0;
  int slot = batched ? 0 : c->single_slot;
  int pieces = batched ? 1 : c->cfg.back_pieces;
  const DevScen* descs = c->d_descs;
  const int4* work = c->d_work + n_fw;
  int n_work = n_tw;
  hipGraphNode_t prev = nullptr;
  hipError_t e = hipSuccess;
  int n_ev = 0;
  auto mark = [&](int kind) {
    if (e != hipSuccess || !profiled) return;
    hipGraphNode_t node;
    e = hipGraphAddEventRecordNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0,
                                   c->gev[n_ev++]);
    prev = node;
    if (kind >= 0) c->gkind.push_back(kind);
  };
  auto add = [&](void* fn, int grid, int block, size_t shmem, void** args) {
    if (e != hipSuccess) return;
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(block);
    kp.sharedMemBytes = (unsigned)shmem;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  };
  // with lane changes, a launch of more tiles than are resident at once
  // starts each XCD's longest-running tiles first, by their times since
  // the last replay (ahead of the events that time the kernels)
  int4* owork = c->d_work + n_fw;
  long long* osnap = c->d_snap + n_fw;
  int on_tw = n_tw;
  if (order_tiles(n_tw)) {
    void* oa[] = {&descs, &owork, &on_tw, &osnap};
    add(order_kernel(), 8, kOrderThreads, 0, oa);
  }
  for (int j = 0; j < kLeadEvents; ++j) mark(-1);
  for (int s = 0; s < K; ++s) {
    int step = s;
    if (n_fw > 0) {
      void* sa[] = {&descs, &fslot, &fwork, &step};
      add(step_kernel(fbatched, skip_lanes(c, n_fw)), n_fw, kWave, 0, sa);
      mark(3);
    }
    if (n_tw > 0) {
      void* fa[] = {&descs, &slot, &work, &pieces, &step};
      add(front_kernel(batched), n_tw, kFrontThreads,
          (size_t)kLcBytesPerWord * c->lc_words, fa);
      mark(0);
      void* ba[] = {&descs, &slot, &work, &n_work, &step};
      add(back_kernel(batched), n_tw + (batched ? 0 : c->n_extra),
          kBackThreadsPerPiece, 0, ba);
      mark(1);
    }
  }
  DevScen* mdescs = c->d_descs;
  const int* list = c->d_list;
  int n = c->n_net, k = K;
  void* aa[] = {&mdescs, &list, &n, &k};
  add(advance_kernel(), (n + 63) / 64, 64, 0, aa);
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, SIM_E_DEVICE, "graph: %s", hipGetErrorString(e));
  *out = ex;
  return SIM_OK;
}

// Replays a profiled graph once and adds its per-kernel times (the graph
// last built with profiled = true).
sim_status run_profiled(sim_ctx* c, hipGraphExec_t ex) {
  HIPCHK(c, hipGraphLaunch(ex, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ev = 0;  // mean cost of one event node
  for (int j = 0; j + 1 < kLeadEvents; ++j) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->gev[j], c->gev[j + 1]));
    ev += ms;
  }
  ev /= (kLeadEvents - 1);
  const int e0 = kLeadEvents - 1;  // the event before the first kernel
  for (size_t j = 0; j < c->gkind.size(); ++j) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->gev[e0 + j], c->gev[e0 + j + 1]));
    c->acc_launches[c->gkind[j]]++;
    c->acc_ms[c->gkind[j]] += std::max(0.0, (double)ms - ev);
  }
  return SIM_OK;
}

// Brackets one launch with a pair of events when profiling is on.
template <class F>
sim_status timed(sim_ctx* c, int kind, F&& launch) {
  if (!c->profile) {
    HIPCHK(c, launch());
    return SIM_OK;
  }
  if (c->events.size() < 2 * (c->n_pairs + 1)) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
    c->event_kind.push_back(0);
  }
  HIPCHK(c, hipEventRecord(c->events[2 * c->n_pairs], c->stream));
  HIPCHK(c, launch());
  HIPCHK(c, hipEventRecord(c->events[2 * c->n_pairs + 1], c->stream));
  c->event_kind[c->n_pairs] = kind;
  ++c->n_pairs;
  return SIM_OK;
}

}  // namespace

extern "C" sim_status sim_profile(sim_ctx* c, int32_t enable) {
  if (!c) return SIM_E_INVAL;
  c->profile = enable != 0;
  return SIM_OK;
}

extern "C" sim_status sim_kernel_times(sim_ctx* c, sim_kernel_time out[4]) {
  if (!c) return SIM_E_INVAL;
  if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (size_t p = 0; p < c->n_pairs; ++p) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->events[2 * p], c->events[2 * p + 1]));
    c->acc_launches[c->event_kind[p]]++;
    c->acc_ms[c->event_kind[p]] += ms;
  }
  c->n_pairs = 0;
  for (int k = 0; k < 4; ++k) {
    out[k] = sim_kernel_time{c->acc_launches[k], c->acc_ms[k]};
    c->acc_launches[k] = 0;
    c->acc_ms[k] = 0;
  }
  return SIM_OK;
}

// The slot list of a step call, checked and split into network and ring
// slots.
static sim_status check_step(sim_ctx* c, const int32_t* slots, int32_t n_slots,
                             int32_t n_steps, std::vector<int32_t>& net,
                             std::vector<int32_t>& ring) {
  if (!c) return SIM_E_INVAL;
  if (!slots || n_slots < 1) return fail(c, SIM_E_INVAL, "no slots");
  if (n_steps < 0) return fail(c, SIM_E_INVAL, "negative step count");
  std::vector<uint8_t> seen(c->slots.size(), 0);
  for (int32_t k = 0; k < n_slots; ++k) {
    sim_status st = check_slot(c, slots[k]);
    if (st != SIM_OK) return st;
    const Slot& S = c->slots[slots[k]];
    if (!S.net || !S.veh) return fail(c, SIM_E_STATE, "slot %d is not loaded", slots[k]);
    if (seen[slots[k]]++) return fail(c, SIM_E_INVAL, "slot %d listed twice", slots[k]);
    if ((int64_t)S.t + n_steps > INT32_MAX - 1)
      return fail(c, SIM_E_CAPACITY, "step index would overflow");
    if (S.fused && (int64_t)S.t + n_steps >= (int64_t)1 << 30)
      return fail(c, SIM_E_CAPACITY, "one-kernel steps stop at t = 2^30");
    (S.ring ? ring : net).push_back(slots[k]);
  }
  return SIM_OK;
}

static sim_status step_body(sim_ctx* c, const int32_t* slots, int32_t n_slots,
                            int32_t n_steps) {
  std::vector<int32_t> net, ring;
  sim_status st = check_step(c, slots, n_slots, n_steps, net, ring);
  if (st != SIM_OK) return st;
  if (n_steps == 0) return SIM_OK;
  st = build_work(c, net, ring);
  if (st != SIM_OK) return st;
  if (!net.empty()) {
    const int K = c->cfg.graph_steps;
    int32_t done = 0;
    if (K > 0 && c->profile) {
      // profiled: graphs with events between the kernels, harvested after
      // every replay (the remainder gets a graph of its own)
      if (n_steps >= K && (!c->pgraph || c->pgraph_k != K)) {
        if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
        c->pgraph = nullptr;
        c->pgraph_k = 0;
        st = build_graph(c, K, true, &c->pgraph);
        if (st != SIM_OK) return st;
        c->pgraph_k = K;
      }
      for (; done + K <= n_steps; done += K) {
        st = run_profiled(c, c->pgraph);
        if (st != SIM_OK) return st;
      }
      if (done < n_steps) {
        // the event kinds belong to the graph built last: rebuild the
        // cached one afterwards
        hipGraphExec_t rg = nullptr;
        st = build_graph(c, n_steps - done, true, &rg);
        if (st != SIM_OK) return st;
        st = run_profiled(c, rg);
        (void)hipGraphExecDestroy(rg);
        if (st != SIM_OK) return st;
        done = n_steps;
        if (c->pgraph) (void)hipGraphExecDestroy(c->pgraph);
        c->pgraph = nullptr;
        c->pgraph_k = 0;
      }
    } else if (K > 0 && n_steps >= K) {
      if (!c->graph || c->graph_k != K) {
        if (c->graph) (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
        st = build_graph(c, K, false, &c->graph);
        if (st != SIM_OK) return st;
        c->graph_k = K;
      }
      for (; done + K <= n_steps; done += K) HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    }
    if (K > 0 && !c->profile && n_steps - done >= kMinRestGraph) {
      // the remainder as a graph of its own, kept for the next call that
      // leaves the same remainder (e.g. repeated windows of a few steps)
      const int R = n_steps - done;
      if (!c->rgraph || c->rgraph_k != R) {
        if (c->rgraph) (void)hipGraphExecDestroy(c->rgraph);
        c->rgraph = nullptr;
        c->rgraph_k = 0;
        st = build_graph(c, R, false, &c->rgraph);
        if (st != SIM_OK) return st;
        c->rgraph_k = R;
      }
      HIPCHK(c, hipGraphLaunch(c->rgraph, c->stream));
      done = n_steps;
    }
    const int32_t rest = n_steps - done;
    const int n_fw = c->n_fwork, n_tw = c->n_work - c->n_fwork;
    for (int32_t s = 0; s < rest; ++s) {
      if (n_fw > 0) {
        st = timed(c, 3, [&] {
          return launch_step(c->d_descs, c->fused_slot, c->d_work, n_fw, s,
                             skip_lanes(c, n_fw), c->stream);
        });
        if (st != SIM_OK) return st;
      }
      if (n_tw > 0) {
        st = timed(c, 0, [&] {
          return launch_front(c->d_descs, c->single_slot, c->d_work + n_fw, n_tw,
                              c->cfg.back_pieces, s, c->lc_words, c->stream);
        });
        if (st != SIM_OK) return st;
        st = timed(c, 1, [&] {
          return launch_back(c->d_descs, c->single_slot, c->d_work + n_fw, n_tw,
                             c->n_extra, s, c->stream);
        });
        if (st != SIM_OK) return st;
      }
    }
    if (rest > 0)
      HIPCHK(c, launch_advance(c->d_descs, c->d_list, c->n_net, rest, c->stream));
  }
  if (!ring.empty()) {
    st = timed(c, 2, [&] {
      return launch_ring(c->d_descs, c->d_list + c->n_net, c->n_ring, n_steps, c->stream);
    });
    if (st != SIM_OK) return st;
  }
  for (int32_t sl : net) c->slots[sl].t += n_steps;
  for (int32_t sl : ring) c->slots[sl].t += n_steps;
  return SIM_OK;
}

// sim_step without any allocation: the work list goes to the device's fixed
// scratch (csrc/scratch.hip) instead of context memory, and every kernel
// is launched directly (no graph is instantiated).
static sim_status step_noalloc_body(sim_ctx* c, const int32_t* slots,
                                    int32_t n_slots, int32_t n_steps) {
  std::vector<int32_t> net, ring;
  sim_status st = check_step(c, slots, n_slots, n_steps, net, ring);
  if (st != SIM_OK) return st;
  if (n_steps == 0) return SIM_OK;
  void* base = scratch_ptr(c->device);
  if (!base) return fail(c, SIM_E_DEVICE, "device scratch not set up");
  WorkPlan wp;
  plan_work(c, net, ring, wp);
  if (wp.work.size() > (size_t)kScratchWork)
    return fail(c, SIM_E_CAPACITY,
                "sim_step_noalloc: %zu tiles, the fixed scratch holds %d",
                wp.work.size(), kScratchWork);
  if (wp.list.size() > (size_t)kScratchSlots)
    return fail(c, SIM_E_CAPACITY,
                "sim_step_noalloc: %zu slots, the fixed scratch holds %d",
                wp.list.size(), kScratchSlots);
  c->nowork.swap(wp.work);
  c->nolist.swap(wp.list);
  int4* d_work = static_cast<int4*>(base);
  int* d_list = reinterpret_cast<int*>(d_work + kScratchWork);
  HIPCHK(c, up(d_work, c->nowork.data(), (int64_t)c->nowork.size(), c->stream));
  HIPCHK(c, up(d_list, c->nolist.data(), (int64_t)c->nolist.size(), c->stream));
  const int n_fw = wp.n_fwork, n_tw = (int)c->nowork.size() - wp.n_fwork;
  if (wp.n_net > 0) {
    for (int32_t s = 0; s < n_steps; ++s) {
      if (n_fw > 0)
        HIPCHK(c, launch_step(c->d_descs, wp.fused_slot, d_work, n_fw, s,
                              skip_lanes(c, n_fw), c->stream));
      if (n_tw > 0) {
        HIPCHK(c, launch_front(c->d_descs, wp.single_slot, d_work + n_fw, n_tw,
                               c->cfg.back_pieces, s, wp.lc_words, c->stream));
        HIPCHK(c, launch_back(c->d_descs, wp.single_slot, d_work + n_fw, n_tw,
                              wp.n_extra, s, c->stream));
      }
    }
    HIPCHK(c, launch_advance(c->d_descs, d_list, wp.n_net, n_steps, c->stream));
  }
  if (wp.n_ring > 0)
    HIPCHK(c, launch_ring(c->d_descs, d_list + wp.n_net, wp.n_ring, n_steps,
                          c->stream));
  for (int32_t sl : net) c->slots[sl].t += n_steps;
  for (int32_t sl : ring) c->slots[sl].t += n_steps;
  return SIM_OK;
}

extern "C" sim_status sim_stats(sim_ctx* c, int32_t slot, sim_stats_t* out) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
  const Slot& S = c->slots[slot];
  if (!S.net || !S.veh) return fail(c, SIM_E_STATE, "slot %d is not loaded", slot);
  unsigned long long h[C_N + 3];
  uint32_t err = 0;
  HIPCHK(c, hipMemsetAsync(c->d_stats, 0, sizeof h, c->stream));
  HIPCHK(c, launch_stats(c->d_descs + slot, c->d_stats, S.ring ? 1 : 0, c->stream));
  HIPCHK(c, hipMemcpyAsync(h, c->d_stats, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&err, S.d.err, sizeof err, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memset(out, 0, sizeof *out);
  out->t = S.t;
  out->veh_updates = (int64_t)h[C_UPDATES];
  out->sum_v = (int64_t)h[C_SUMV];
  out->crossings = (int64_t)h[C_CROSS];
  out->exits = (int64_t)h[C_EXITS];
  out->lane_changes = (int64_t)h[C_LC];
  out->insertions = (int64_t)h[C_INS];
  out->c_occ = (int64_t)h[C_COCC];
  out->n_active = (int64_t)h[C_N];
  out->hash = h[C_N + 1];
  out->n_waiting = (int64_t)h[C_N + 2];
  out->n_arrived = S.n_veh - out->n_active - out->n_waiting;
  out->dev_err = err;
  if (err) return fail(c, SIM_E_DEVICE, "device error bits 0x%x", err);
  return SIM_OK;
}

static sim_status read_state_body(sim_ctx* c, int32_t slot, int8_t* status,
                                  int32_t* link, int8_t* lane, int32_t* x,
                                  int8_t* v, int32_t* rptr, int32_t* exit_t) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  const Slot& S = c->slots[slot];
  if (!S.net || !S.veh) return fail(c, SIM_E_STATE, "slot %d is not loaded", slot);
  const int64_t n = S.n_veh;
  const ExportBufs& o = S.exp;  // staging in the slot's workspace
  hipError_t e = launch_export(c->d_descs + slot, o, (int)n, S.n_links, S.n_lanes,
                               S.ring ? 1 : 0, c->stream);
  const char* what = "export kernels";
  auto down = [&](void* dst, const void* src, size_t b, const char* name) {
    if (e == hipSuccess && dst && b) {
      e = hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, c->stream);
      what = name;
    }
  };
  down(status, o.status, n, "copy status");
  down(link, o.link, 4 * n, "copy link");
  down(lane, o.lane, n, "copy lane");
  down(x, o.x, 4 * n, "copy x");
  down(v, o.v, n, "copy v");
  down(rptr, o.rptr, 4 * n, "copy rptr");
  if (!S.ring) down(exit_t, S.d.exit_t, 4 * (size_t)S.n_route, "copy exit_t");
  if (e == hipSuccess) {
    e = hipStreamSynchronize(c->stream);
    what = "synchronize";
  }
  if (e != hipSuccess)
    return fail(c, SIM_E_DEVICE, "read_state: %s: %s", what, hipGetErrorString(e));
  return SIM_OK;
}

static sim_status link_costs_body(sim_ctx* c, int32_t slot, float* out) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  const Slot& S = c->slots[slot];
  if (!S.net) return fail(c, SIM_E_STATE, "slot %d has no network", slot);
  if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
  std::fill(out, out + S.n_links, 0.0f);
  // cycles of each tile of both sub-steps, shared out over its links by cells
  for (int pass = 0; pass < 2; ++pass) {
    // move-tile counters sit at the entry of each tile's first lane (the
    // tiles may have been rebalanced); they are credited to the static tile
    // holding that lane.  Lane-change tiles use one entry per tile.
    const std::vector<int2>& tiles = pass == 0 ? S.tiles : S.ftiles;
    const size_t entries = pass == 0 ? (size_t)S.n_lanes : tiles.size();
    std::vector<long long> ctr(entries * C_N);
    HIPCHK(c, hipMemcpyAsync(ctr.data(), pass == 0 ? S.d.tile_ctr : S.d.ftile_ctr,
                             sizeof(long long) * ctr.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t t = 0; t < tiles.size(); ++t) {
      const int2 tl = tiles[t];
      double cyc = 0;
      if (pass == 0) {
        for (int32_t q = tl.x; q < tl.x + tl.y; ++q) cyc += (double)ctr[(size_t)q * C_N + C_CYCLES];
      } else {
        cyc = (double)ctr[t * C_N + C_CYCLES];
      }
      const int32_t l0 = (int32_t)(std::upper_bound(S.lane0.begin(), S.lane0.end(), tl.x) -
                                   S.lane0.begin()) - 1;
      double cells = 0;
      int32_t l1 = l0;
      while (l1 < S.n_links && S.lane0[l1] < tl.x + tl.y) {
        cells += (double)S.len[l1] * S.lanes[l1];
        ++l1;
      }
      for (int32_t lk = l0; lk < l1; ++lk)
        out[S.ext_of[lk]] += (float)(cells > 0 ? cyc * S.len[lk] * S.lanes[lk] / cells : 0);
    }
  }
  return SIM_OK;
}

extern "C" sim_status sim_tiling_info(const sim_ctx* cc, int32_t slot, sim_tiling* out) {
  sim_ctx* c = const_cast<sim_ctx*>(cc);
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  if (!out) return fail(c, SIM_E_INVAL, "out is NULL");
  const Slot& S = c->slots[slot];
  if (!S.net) return fail(c, SIM_E_STATE, "slot %d has no network", slot);
  *out = S.tiling;
  return SIM_OK;
}

extern "C" sim_status sim_unload(sim_ctx* c, int32_t slot) {
  sim_status st = check_slot(c, slot);
  if (st != SIM_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->slots[slot] = Slot();
  ++c->slot_gen[slot];
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// The entry points that build host tables: a C++ exception (host memory
// exhausted) becomes an error status instead of crossing the C boundary.

namespace {

template <class F>
sim_status guarded(const sim_ctx* cc, F&& body) {
  sim_ctx* c = const_cast<sim_ctx*>(cc);
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(c, SIM_E_CAPACITY, "host memory exhausted");
  } catch (const std::exception& e) {
    return fail(c, SIM_E_INVAL, "%s", e.what());
  }
}

}  // namespace

extern "C" sim_status sim_create(const sim_config* cfg, sim_ctx** out) {
  return guarded(nullptr, [&] { return create_body(cfg, out); });
}

extern "C" sim_status sim_footprint(const sim_ctx* cc, const sim_params* p,
                                    const sim_network* net,
                                    const sim_vehicles* veh, uint64_t* bytes) {
  return guarded(cc, [&] { return footprint_body(cc, p, net, veh, bytes); });
}

extern "C" sim_status sim_load_network(sim_ctx* c, int32_t slot,
                                       const sim_params* p,
                                       const sim_network* net, void* dev_ws,
                                       uint64_t ws_bytes) {
  return guarded(c, [&] {
    return load_network_body(c, slot, p, net, dev_ws, ws_bytes);
  });
}

extern "C" sim_status sim_load_vehicles(sim_ctx* c, int32_t slot,
                                        const sim_vehicles* v) {
  return guarded(c, [&] { return load_vehicles_body(c, slot, v); });
}

extern "C" sim_status sim_step(sim_ctx* c, const int32_t* slots, int32_t n_slots,
                               int32_t n_steps) {
  return guarded(c, [&] { return step_body(c, slots, n_slots, n_steps); });
}

extern "C" sim_status sim_step_noalloc(sim_ctx* c, const int32_t* slots,
                                       int32_t n_slots, int32_t n_steps) {
  return guarded(c, [&] { return step_noalloc_body(c, slots, n_slots, n_steps); });
}

extern "C" sim_status sim_read_state(sim_ctx* c, int32_t slot, int8_t* status,
                                     int32_t* link, int8_t* lane, int32_t* x,
                                     int8_t* v, int32_t* rptr, int32_t* exit_t) {
  return guarded(c, [&] {
    return read_state_body(c, slot, status, link, lane, x, v, rptr, exit_t);
  });
}

extern "C" sim_status sim_link_costs(sim_ctx* c, int32_t slot, float* out) {
  return guarded(c, [&] { return link_costs_body(c, slot, out); });
}
