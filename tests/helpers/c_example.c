/* c_example.c -- the C ABI of libtransims from plain C: a two-link road,
   two travellers, twenty steps.  Build against the library and the HIP
   runtime, e.g.
     gcc -std=c11 -D__HIP_PLATFORM_AMD__ -I include -I /opt/rocm/include \
         c_example.c -L paper_cs_0105004_amd -ltransims -L /opt/rocm/lib \
         -lamdhip64
   The tests build it against a host-only copy of the library. */
#include <stdint.h>
#include <stdio.h>

#include <hip/hip_runtime_api.h>

#include "transims.h"

#define CHECK(call)                                                      \
  do {                                                                   \
    sim_status st_ = (call);                                             \
    if (st_ != SIM_OK) {                                                 \
      fprintf(stderr, "%s: %d (%s)\n", #call, (int)st_,                   \
              sim_last_error(ctx));                                      \
      return 1;                                                          \
    }                                                                    \
  } while (0)

int main(void) {
  /* node 0 -> node 1 -> node 2: a 2-lane link of 30 cells, then a 1-lane
     link of 30 cells (lane 0 is the leftmost) */
  const int32_t from[2] = {0, 1}, to[2] = {1, 2}, len[2] = {30, 30};
  const int8_t lanes[2] = {2, 1}, rank[2] = {0, 0};
  const double xy[6] = {0, 0, 1, 0, 2, 0};
  sim_network net = {0};
  net.n_nodes = 3;
  net.n_links = 2;
  net.from = from;
  net.to = to;
  net.len = len;
  net.lanes = lanes;
  net.rank = rank;
  net.node_xy = xy;

  /* two travellers along links 0 then 1, leaving parking at steps 0, 1 */
  const int32_t depart[2] = {0, 1}, route_links[4] = {0, 1, 0, 1};
  const int64_t route_off[3] = {0, 2, 4};
  sim_vehicles veh = {0};
  veh.n = 2;
  veh.depart = depart;
  veh.route_off = route_off;
  veh.route_links = route_links;

  sim_params p = {0};
  p.flags = SIM_FLAG_LANE_CHANGE;
  p.vmax = 5;
  p.slow_thr = 858993459u; /* floor(0.2 * 2^32) */
  p.lc_thr = (uint64_t)1 << 32; /* always take a lane change that pays */
  p.lc_desp = 10;
  p.seed = 42;

  sim_ctx* ctx = NULL;
  sim_config cfg = {0}; /* zero fields: library defaults */
  cfg.abi_version = SIM_ABI_VERSION;
  cfg.max_slots = 1;
  cfg.stream = NULL; /* the default stream */
  CHECK(sim_create(&cfg, &ctx));

  uint64_t bytes = 0;
  CHECK(sim_footprint(ctx, &p, &net, &veh, &bytes));
  void* ws = NULL; /* the workspace belongs to the caller */
  if (hipMalloc(&ws, bytes) != hipSuccess) return 1;
  CHECK(sim_load_network(ctx, 0, &p, &net, ws, bytes));
  CHECK(sim_load_vehicles(ctx, 0, &veh));

  const int32_t slot = 0;
  CHECK(sim_step(ctx, &slot, 1, 20)); /* enqueues; sim_stats waits */
  sim_stats_t st;
  CHECK(sim_stats(ctx, 0, &st));
  int32_t exit_t[4];
  CHECK(sim_read_state(ctx, 0, NULL, NULL, NULL, NULL, NULL, NULL, exit_t));
  printf("t %d, active %lld, arrived %lld, vehicle-updates %lld\n", st.t,
         (long long)st.n_active, (long long)st.n_arrived,
         (long long)st.veh_updates);

  CHECK(sim_unload(ctx, 0));
  hipFree(ws);
  CHECK(sim_destroy(ctx));
  return 0;
}
