/*
 * transims.h -- C ABI of libtransims, the MI355X (gfx950) implementation of
 * the per-second cellular-automaton update of the TRANSIMS micro-simulation
 * (K. Nagel, M. Rickert, "Parallel implementation of the TRANSIMS
 * micro-simulation").
 *
 * One step moves every vehicle on every link of a scenario by one second
 * (Section "Microsimulation driving logic"): 7.5 m cells holding at most one
 * vehicle, integer speeds 0..vmax cells per step, accelerate / brake to the
 * gap / random slowdown / move (rules i-iii), a lane-change sub-step before
 * the forward move, unsignalised intersections with priority (the minor
 * approach yields to the priority link), and vehicles entering from and
 * exiting to parking along precomputed routes.  The update order follows
 * the paper's per-step sequence: lane-change sub-step, boundary exchange,
 * velocity-and-move sub-step, boundary exchange (Section "Micro-simulation
 * parallelization: Domain decomposition"); on one GPU the two boundary
 * exchanges become kernel boundaries plus in-memory handoff slots.
 *
 * Rules the paper leaves open are fixed as follows (the same readings bind
 * every implementation that claims to compute this step):
 *   - speeds: v1 = min(v+1, vmax); v2 = min(v1, gap); v3 = v2-1 when v2 > 0
 *     and the vehicle's draw u < slow_thr, else v2; x' = x + v3;
 *   - draws: word 0 of Philox4x32-10 under key (seed lo, seed hi) at counter
 *     (vehicle id, t, sub-step, 0), sub-step 0 = lane change, 1 = slowdown;
 *   - parking: at most one vehicle per link per step enters cell 0 of the
 *     lowest lane whose cell 0 is empty, FIFO by (depart, id);
 *   - lane change: incentive + gap checks of vmax cells; turn lanes shrink
 *     the accepted gap toward the node; two movers into one cell: the one
 *     from the lower lane moves;
 *   - intersections: the lead vehicle of a lane within vmax cells of the
 *     node aims at lane min(k, lanes'-1) of its next link; per target lane
 *     the smallest (rank, lane) wins and may drive min(vmax, x_rear) cells
 *     into the next link; losers stop at the link end; a trip ends at the
 *     end of the last link (extra = vmax).
 * Every step is integer; results are bit-identical to the CPU oracle.
 *
 * Threading: a context is driven by one host thread.  The one exception is
 * loading: sim_load_network and sim_load_vehicles may run on other threads
 * at the same time as the driving thread's calls, for slots that no
 * concurrent call names (a serving loop loads new scenarios while the slots
 * already running keep stepping).  A load makes the context's device
 * current on its thread.  All device work of a context runs on the stream
 * given at creation.  No exception crosses this boundary.
 */
#ifndef TRANSIMS_H
#define TRANSIMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 3

typedef enum {
  SIM_OK = 0,
  SIM_E_INVAL = -1,    /* invalid argument or inconsistent input data        */
  SIM_E_NOMEM = -2,    /* the caller's workspace is smaller than needed      */
  SIM_E_STATE = -3,    /* wrong call order, or slot not loaded               */
  SIM_E_DEVICE = -4,   /* HIP runtime error, or sticky device error bits     */
  SIM_E_CAPACITY = -5, /* a size exceeds a library limit, or host memory ran
                          out (no C++ exception crosses this interface)     */
  SIM_E_ABI = -6       /* abi_version mismatch                               */
} sim_status;

/* scenario flags */
#define SIM_FLAG_RING 1u        /* one periodic lane, no nodes, no parking    */
#define SIM_FLAG_LANE_CHANGE 2u /* lane-change sub-step on multi-lane links   */
#define SIM_FLAG_TURN_LANES 4u  /* lane changes toward the lanes of the turn  */

/* device error bits reported in sim_stats_t.dev_err */
#define SIM_DEVERR_LANE_FULL 1u /* a lane received more vehicles than cells   */

typedef struct sim_ctx sim_ctx;

typedef struct {
  int32_t abi_version; /* must be SIM_ABI_VERSION                           */
  int32_t max_slots;   /* number of independent scenario slots (>= 1)       */
  void* stream;        /* hipStream_t for all device work; NULL = default   */
  int32_t tile_lanes;   /* lanes per workgroup tile (whole links), 1..64;
                           0 = default (16; 32 for scenarios with lane
                           changes)                                         */
  int32_t back_pieces;  /* wavefronts per tile in the move sub-step, which
                           share the tile's lanes by vehicle load, 1..8;
                           0 = default (4)                                  */
  int32_t graph_steps;  /* steps per HIP graph replay in sim_step, at most
                           4096; 0 = default (64); < 0 = launch kernels one
                           by one.  Steps left after whole replays (or a
                           call of fewer steps) run as a graph of their own
                           when there are at least 8 of them; that graph is
                           kept while later calls leave the same number.
                           With lane changes and more tiles than are
                           resident at once, each replay first reorders the
                           tiles by their measured lane-change time, which
                           changes no result                               */
  int32_t step_mode;    /* 0 = one kernel per step for scenarios without
                           lane changes whose links all have >= 2*vmax
                           cells, two kernels (lane-change / move sub-step)
                           otherwise; 1 = always two kernels; 2 = as 0, and
                           the one-kernel step skips lanes that are empty and
                           stay empty (less memory traffic, one more round of
                           dependent loads).  Results are the same in every
                           mode.                                            */
  int32_t tile_cells;   /* one-kernel step, and scenarios with lane
                           changes: a tile also stops at this many cells
                           (len x lanes; a longer link is a tile of its
                           own), 64..65536; 0 = default (1024; 4096 for
                           scenarios with lane changes)                     */
  int32_t reserved;     /* must be 0                                        */
} sim_config;

/* Per-scenario parameters. */
typedef struct {
  uint32_t flags;
  int32_t vmax;      /* 1..7 cells per step (5 = 135 km/h)                   */
  uint64_t slow_thr; /* slowdown iff draw < slow_thr; floor(p*2^32), <= 2^32 */
  uint64_t lc_thr;   /* discretionary lane change iff draw < lc_thr, <= 2^32 */
  int32_t lc_desp;   /* desperation distance D (cells) for turn lanes, >= 1  */
  uint64_t seed;     /* Philox key                                          */
} sim_params;

/* Road network, borrowed for the duration of the call (copied). */
typedef struct {
  int32_t n_nodes;
  int32_t n_links;
  const int32_t* from;  /* [n_links] upstream node                         */
  const int32_t* to;    /* [n_links] downstream node (!= from)              */
  const int32_t* len;   /* [n_links] cells; vmax+1..32767 (ring: 1..32767) */
  const int8_t* lanes;  /* [n_links] 1..4; lane 0 is the leftmost          */
  const int8_t* rank;   /* [n_links] 0..127, priority among the links that
                           enter one node (0 first); unique per node        */
  /* lane connectivity, needed with SIM_FLAG_TURN_LANES, else may be NULL:
     entries conn_off[l]..conn_off[l+1]-1 name an out-link of to[l] and the
     lanes [lo, hi] of l from which that turn is made                       */
  const int64_t* conn_off;
  const int32_t* conn_out;
  const int8_t* conn_lo;
  const int8_t* conn_hi;
  const double* node_xy;   /* optional [2*n_nodes]; used only for tiling     */
  const float* link_cost;  /* optional [n_links] tiling weights (e.g. costs
                              measured by sim_link_costs on an earlier run):
                              they weight the ORB cuts, and a tile also
                              stops at the mean weight of the tiles the
                              lane and cell caps alone would make (Section
                              "Adaptive Load Balancing"); each finite and
                              >= 0, else SIM_E_INVAL                        */
  /* optional fixed-time signals at the downstream end of links (Section
     "Microsimulation driving logic": while the light is red a virtual
     vehicle of speed zero stands at the end of the lane).  signal_plan[l]
     is -1 or a plan index j < n_plans (1..63); plan j is red at step t iff
     (t + plan_offset[j]) mod plan_cycle[j] < plan_red[j], cycle >= 1,
     0 <= red <= cycle, offset >= 0.  While red, a lane's lead vehicle
     neither crosses the node nor ends its trip there.  NULL = none.        */
  const int8_t* signal_plan;
  int32_t n_plans;
  const int32_t* plan_cycle;
  const int32_t* plan_red;
  const int32_t* plan_offset;
} sim_network;

/* Travellers and their plans, borrowed for the duration of the call.
   Vehicle id = index.  A vehicle whose status is WAITING enters from parking
   at the first link of its route at step depart or later. */
typedef struct {
  int32_t n;
  const int32_t* depart;      /* [n]                                        */
  const int64_t* route_off;   /* [n+1]; NULL in ring mode                   */
  const int32_t* route_links; /* [route_off[n]]; consecutive links connect  */
  /* optional initial state; all NULL = every vehicle WAITING              */
  const int8_t* init_status;  /* 0 WAITING, 1 ACTIVE, 2 ARRIVED             */
  const int8_t* init_lane;    /* ACTIVE: lane                               */
  const int32_t* init_x;      /* ACTIVE: cell                               */
  const int8_t* init_v;       /* ACTIVE: speed 0..vmax                      */
  const int32_t* init_rptr;   /* ACTIVE: route index of the current link    */
  const int32_t* exit_t0;     /* [route_off[n]] or NULL (= all -1)          */
  int32_t t0;                 /* index of the first step                    */
} sim_vehicles;

typedef struct {
  int32_t t; /* index of the next step                                      */
  int32_t reserved;
  int64_t n_waiting, n_active, n_arrived;
  int64_t veh_updates;  /* sum over steps of vehicles moved               */
  int64_t sum_v;        /* sum over all updates of the new speed           */
  int64_t crossings;    /* moves onto the next link of a route             */
  int64_t exits;        /* trips ended                                     */
  int64_t lane_changes;
  int64_t insertions;
  int64_t c_occ;        /* sum over steps of cells in lanes holding a car  */
  uint64_t hash;        /* order-independent hash of the current state     */
  uint32_t dev_err;     /* SIM_DEVERR_* bits                               */
  uint32_t reserved2;
} sim_stats_t;

/* Creates a context on the current HIP device.  *out receives it.
   Passage: the whole simulated region advanced as one unit per time step
   (Section "Micro-simulation parallelization: Domain decomposition"; on
   one GPU the domains become the workgroup tiles of each loaded slot).
   cfg is read during the call only.  The context owns its host memory and
   a small device area (scenario descriptors, counter staging); release it
   with sim_destroy.  The configuration is checked before any device call:
   a field out of its stated range returns SIM_E_INVAL, another abi_version
   SIM_E_ABI; on any error *out is NULL. */
sim_status sim_create(const sim_config* cfg, sim_ctx** out);

/* Bytes of device workspace that sim_load_network + sim_load_vehicles need
   for this scenario (the caller allocates them, e.g. as a torch tensor).
   Passage: the state the driving logic updates -- 7.5 m cells of every lane
   of every link, and the travellers' plans (Sections "Microsimulation
   driving logic" and "Introduction"); memory is sized per scenario, as the
   paper sizes each CPU's domain by its share of links (Section "Graph
   partitioning").  veh may be NULL (network part only).  Inputs are
   borrowed for the call and checked as in the loaders: SIM_E_INVAL on bad
   input, SIM_E_CAPACITY if a count exceeds a library limit.  ctx may be
   NULL (default configuration). */
sim_status sim_footprint(const sim_ctx* ctx, const sim_params* p,
                         const sim_network* net, const sim_vehicles* veh,
                         uint64_t* bytes);

/* Loads a network into `slot`, tiling its links onto workgroups (orthogonal
   recursive bisection over link midpoints, weighted by cells or by
   net->link_cost).  Passage: links of lanes of 7.5 m cells meeting at
   nodes (Section "Microsimulation driving logic") and their partitioning
   by orthogonal bisection (Section "Graph partitioning"); links are never
   split here (one GPU holds every tile).  Every array of net is borrowed
   for the call and copied; p gives vmax, slow_thr, lc_thr, lc_desp, seed
   and flags.  dev_ws is device memory owned by the caller that must
   stay valid until sim_unload; the library never frees it.  Any scenario
   previously in the slot is unloaded, also when the call fails. */
sim_status sim_load_network(sim_ctx* ctx, int32_t slot, const sim_params* p,
                            const sim_network* net, void* dev_ws,
                            uint64_t ws_bytes);

/* Loads vehicles and routes into a slot holding a network. Synchronises the
   context stream before returning. Passage: each traveller's plan, a route
   through the network fixed before the simulation (Section "Introduction"),
   executed by entering from parking at the route's first link and exiting to
   parking at its last (Sections "Microsimulation driving logic" and "Micro-
   simulation parallelization: Domain decomposition"). The arrays of v are
   borrowed for the call and copied; an optional initial state restarts a
   saved run at step v->t0. The routes also set the order in which each XCD's
   tiles are launched: heaviest first by planned load (the routes using a
   link times its cells), which shortens a launch's tail and leaves every
   result unchanged. The input is checked on the host (route_off starts at 0
   and rises strictly, routes connect, placements fit) before it is used; on
   any error the slot holds no vehicles and must be loaded again before it is
   stepped. */
sim_status sim_load_vehicles(sim_ctx* ctx, int32_t slot,
                             const sim_vehicles* veh);

/* Enqueues n_steps steps of every listed slot on the context stream and
   returns without waiting.  The slots advance together in one launch per
   sub-step; they never interact.  Passage: one step is one second of
   traffic (Section "Microsimulation driving logic": rules i-iii, lane
   changing, intersections) in the per-step order lane change, exchange,
   speed and move, exchange (Section "Micro-simulation parallelization:
   Domain decomposition"); parking adds no exchange.  slots is borrowed for
   the call.  Errors (before anything is enqueued): SIM_E_INVAL for an
   empty or repeated slot list, SIM_E_STATE for a slot without vehicles,
   SIM_E_CAPACITY when t would overflow, SIM_E_DEVICE for a failed launch.
   Device-side errors surface in the next sim_stats. */
sim_status sim_step(sim_ctx* ctx, const int32_t* slots, int32_t n_slots,
                    int32_t n_steps);

/* sim_step for callers that cannot allocate device memory: code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc.
   Same arguments, semantics and results as sim_step, but it calls no
   hipMalloc, hipFree or other allocating routine and instantiates no
   graph: the call's work list (one entry per workgroup tile of the listed
   slots) is copied into a fixed device scratch array of the library, at
   most 131,072 tiles and 16,384 slots per call (2.1 MiB, held on each GPU
   the library runs on until the process ends), and every kernel is
   launched directly on the context stream.  A call beyond those limits
   returns SIM_E_CAPACITY before enqueuing anything.  Every call on one GPU
   shares that array: calls on one stream are ordered, but calls that
   overlap on different streams of the same GPU race and must not be
   issued.  Host arrays are borrowed for the call. */
sim_status sim_step_noalloc(sim_ctx* ctx, const int32_t* slots,
                            int32_t n_slots, int32_t n_steps);

/* Waits for the stream and reports the slot's counters and state hash.
   Passage: the inputs of the real-time ratio, simulated seconds over wall
   time per step (Section "Performance prediction for the TRANSIMS
   micro-simulation"), and of the per-step load the paper monitors (Section
   "Adaptive Load Balancing"): steps taken, vehicles moved, crossings.  out
   is written by the call.  Returns SIM_E_STATE for an unloaded slot and
   SIM_E_DEVICE (with out filled) if device error bits are set. */
sim_status sim_stats(sim_ctx* ctx, int32_t slot, sim_stats_t* out);

/* Waits for the stream and copies the per-vehicle state to host arrays of
   n entries (any may be NULL): status, link (-1 unless ACTIVE), lane, x, v,
   rptr; exit_t receives route_off[n] entries.  Passage: the vehicle state
   of the cellular automaton -- cell, lane and integer speed (Section
   "Microsimulation driving logic") -- and the step at which each vehicle
   left each link of its plan, the link travel times the iteration between
   runs feeds back (Section "Introduction").  Host arrays are owned by the
   caller.  Errors: SIM_E_STATE for an unloaded slot, SIM_E_DEVICE if a
   copy fails.  The export goes through a staging area of 15 bytes per
   vehicle in the slot's workspace (sim_footprint counts it), so the call
   allocates nothing. */
sim_status sim_read_state(sim_ctx* ctx, int32_t slot, int8_t* status,
                          int32_t* link, int8_t* lane, int32_t* x, int8_t* v,
                          int32_t* rptr, int32_t* exit_t);

/* Waits for the stream and reports the measured cost per link (device
   clock cycles spent on the link's tile since the vehicles were loaded,
   shared out by cells), for use as net->link_cost of a later run: the
   paper's adaptive load balancing, which re-partitions by the load measured
   in the run before.  out has n_links entries, in the caller's link order. */
sim_status sim_link_costs(sim_ctx* ctx, int32_t slot, float* out);

typedef struct {
  int32_t n_tiles;
  int32_t n_lanes;
  int64_t n_cells;
  double e_dmn;      /* mean / max tile weight over the 8 XCD domains      */
  double e_tile;     /* mean / max weight over tiles                       */
} sim_tiling;

/* The decomposition of the slot's network into workgroup tiles and its
   balance: e_dmn is the paper's partition efficiency (Section "Graph
   partitioning": the load of an ideal split over the load of the largest
   part), taken over the 8 XCDs; e_tile is the same over the tiles. */
sim_status sim_tiling_info(const sim_ctx* ctx, int32_t slot, sim_tiling* out);

/* Kernel timing (the paper monitors the time per step, Section "Adaptive
   Load Balancing"): while enabled, sim_step runs its steps as HIP graphs
   with an event node before the first kernel and after every kernel, and
   with eight back-to-back event nodes ahead of them; a kernel's time is the
   interval between the events around it less the mean interval between two
   back-to-back events of the same replay (the cost of an event node
   itself).  With graph_steps < 0, and for the ring kernel, each launch is
   bracketed by two events on the context stream instead (no correction).
   sim_kernel_times waits for the stream, reports per kernel kind (0 = front
   / lane-change sub-step, 1 = back / move sub-step, 2 = ring, 3 = one-kernel
   step) the number of launches and their summed duration, and resets the
   sums. */
typedef struct {
  int64_t launches;
  double total_ms;
} sim_kernel_time;

sim_status sim_profile(sim_ctx* ctx, int32_t enable);
sim_status sim_kernel_times(sim_ctx* ctx, sim_kernel_time out[4]);

/* Forgets the slot (its workspace may then be released by the caller).
   Passage: the end of one run of an iteration series (Section "Adaptive
   Load Balancing": the next run starts again from the plans).  Waits for
   the stream first.  SIM_E_INVAL for a slot out of range. */
sim_status sim_unload(sim_ctx* ctx, int32_t slot);

/* Destroys the context and its library-owned device and host memory.
   No passage of the paper: resource release only.  Waits for the stream;
   caller workspaces are never freed.  SIM_E_INVAL for NULL. */
sim_status sim_destroy(sim_ctx* ctx);

/* Text of the last error on this context ("" if none); owned by the
   context, valid until its next call.  No passage of the paper: error
   reporting only. */
const char* sim_last_error(const sim_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
