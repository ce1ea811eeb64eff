/*
 * transims_oracle.h -- CPU oracle for the TRANSIMS cellular-automaton step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of the per-second update described in Nagel & Rickert,
 * "Parallel implementation of the TRANSIMS micro-simulation" (Section
 * "Microsimulation driving logic" and the update sequence of Section
 * "Micro-simulation parallelization: Domain decomposition").  It exists to
 * check the GPU library against; only the tests, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every rule the paper leaves open is fixed by the readings listed at the top
 * of transims_oracle.c; the GPU library follows the same readings.
 */
#ifndef TRANSIMS_ORACLE_H
#define TRANSIMS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_FLAG_RING 1u        /* single periodic lane, no nodes            */
#define ORC_FLAG_LANE_CHANGE 2u /* sub-step 1: sideways moves                */
#define ORC_FLAG_TURN_LANES 4u  /* lane-change toward the lanes of the turn  */

#define ORC_WAITING 0
#define ORC_ACTIVE 1
#define ORC_ARRIVED 2

typedef struct {
  uint32_t flags;
  int32_t vmax;      /* 1..7 cells per step                                  */
  uint64_t slow_thr; /* random slowdown iff draw < slow_thr (0..2^32)        */
  uint64_t lc_thr;   /* discretionary change accepted iff draw < lc_thr      */
  int32_t lc_desp;   /* desperation distance D in cells (mandatory changes)  */
  uint64_t seed;     /* Philox key = (seed low word, seed high word)         */
} orc_params;

typedef struct {
  int32_t n_nodes;
  int32_t n_links;
  const int32_t* from;  /* [n_links] */
  const int32_t* to;    /* [n_links] */
  const int32_t* len;   /* [n_links] cells, >= vmax+1                         */
  const int8_t* lanes;  /* [n_links] 1..4, lane 0 = leftmost                 */
  const int8_t* rank;   /* [n_links] priority among links into `to`, 0 first */
  /* lane connectivity (used with ORC_FLAG_TURN_LANES only):
     for link l, entries conn_off[l]..conn_off[l+1]-1 give an out-link of
     to[l] and the lanes [lo, hi] of l from which that turn is made.        */
  const int64_t* conn_off; /* [n_links+1] or NULL */
  const int32_t* conn_out;
  const int8_t* conn_lo;
  const int8_t* conn_hi;
  /* fixed-time signals at the downstream end of links (reading S1-S3):
     signal_plan[l] = -1 (none) or a plan index; plan j is red at step t iff
     (t + plan_offset[j]) mod plan_cycle[j] < plan_red[j].  NULL = none.    */
  const int8_t* signal_plan; /* [n_links] or NULL */
  int32_t n_plans;
  const int32_t* plan_cycle; /* [n_plans], >= 1               */
  const int32_t* plan_red;   /* [n_plans], 0..cycle           */
  const int32_t* plan_offset;/* [n_plans], >= 0               */
} orc_network;

typedef struct {
  int32_t n;
  const int32_t* depart;      /* [n] */
  const int64_t* route_off;   /* [n+1] (NULL in ring mode) */
  const int32_t* route_links; /* [route_off[n]] */
  /* optional initial state (all NULL = every vehicle WAITING)              */
  const int8_t* init_status;  /* ORC_WAITING / ORC_ACTIVE / ORC_ARRIVED    */
  const int8_t* init_lane;
  const int32_t* init_x;
  const int8_t* init_v;
  const int32_t* init_rptr;   /* route index of the current link           */
  const int32_t* exit_t0;     /* [route_off[n]] or NULL (= all -1)         */
  int32_t t0;                 /* first step index                          */
} orc_vehicles;

typedef struct {
  int32_t t;
  int64_t n_waiting, n_active, n_arrived;
  int64_t veh_updates; /* sum over steps of active vehicles moved          */
  int64_t sum_v;       /* sum over all updates of the new velocity         */
  int64_t crossings;   /* moves onto the next link of the route            */
  int64_t exits;       /* moves off the last link (trip ends)              */
  int64_t lane_changes;
  int64_t insertions;
  int64_t c_occ;       /* sum over steps of cells in lanes holding a car   */
  uint64_t hash;       /* order-independent hash of the current state      */
} orc_stats;

typedef struct orc_sim orc_sim;

/* Returns NULL on invalid input, with a message in err. */
orc_sim* orc_create(const orc_params* p, const orc_network* net,
                    const orc_vehicles* veh, char* err, int errlen);
void orc_destroy(orc_sim* s);
/* Advances n steps.  Returns 0, or -1 if an internal invariant broke. */
int orc_step(orc_sim* s, int32_t n);
void orc_get_stats(const orc_sim* s, orc_stats* out);
/* Per-vehicle state; link = -1, lane = x = v = 0 when not active.
   exit_t receives route_off[n] entries (may be NULL). */
void orc_get_state(const orc_sim* s, int8_t* status, int32_t* link,
                   int8_t* lane, int32_t* x, int8_t* v, int32_t* rptr,
                   int32_t* exit_t);

/* Philox4x32-10 and its 4x64 sibling (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]);
/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z);

#ifdef __cplusplus
}
#endif
#endif
