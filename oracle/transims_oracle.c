/*
 * transims_oracle.c -- CPU oracle for the TRANSIMS cellular-automaton step.
 *
 * TEST INFRASTRUCTURE ONLY (see transims_oracle.h).  Plain, single-threaded,
 * arrays indexed by (link, lane, cell); no blocking, no fusion.  Each step
 * follows the paper's order: vehicles leave parking, lanes are changed in the
 * first sub-step, speeds are computed and vehicles moved in the second
 * (Section "Microsimulation driving logic"; update sequence in Section
 * "Micro-simulation parallelization: Domain decomposition").
 *
 * Readings of what the paper leaves open (the GPU library uses the same):
 *  R1  Car following (rules i-iii of the driving-logic section) is the
 *      Nagel-Schreckenberg order: v1 = min(v+1, vmax); v2 = min(v1, gap);
 *      v3 = v2-1 if v2 > 0 and the vehicle's draw u < slow_thr, else v2;
 *      x' = x + v3.  gap = empty cells to the vehicle ahead.  "Velocity
 *      proportional to the distance" with a 1 s step reads as v <= gap.
 *  R2  All updates inside a sub-step are synchronous: every vehicle reads the
 *      state left by the previous sub-step (locality, Section "parallel-
 *      ization": state t+1 depends only on state t).
 *  R3  Randomness: Philox4x32-10, key = (seed lo, seed hi), counter =
 *      (vehicle id, t, sub-step, 0), word 0 of the output.  Sub-step 0 is the
 *      lane-change draw, 1 the slowdown draw.  p enters only as the integer
 *      threshold slow_thr = floor(p * 2^32), computed exactly on the host.
 *  R4  Ring mode: one periodic lane of L cells; gap is measured cyclically;
 *      a lone vehicle sees gap L-1.
 *  R5  Vehicles leave parking and enter the network
 *      at cell 0 of the first route link, into the lowest lane whose cell 0
 *      is empty, with v = 0; per link a FIFO ordered by (depart, id); at most
 *      one per link per step; a blocked head blocks the queue.
 *  R6  Lane change (first sub-step), on links with >= 2 lanes:
 *        ahead(m)  = empty cells in lane m from x+1 up to the first vehicle
 *                    or the link end, capped at vmax;
 *        behind(m) = empty cells in lane m from x-1 back to the first
 *                    vehicle, capped at vmax; cells before the link start
 *                    count as empty;
 *        the cell (m, x) must be empty.
 *      With turn lanes, a vehicle outside the lanes [lo, hi] of its next
 *      turn must move one lane toward them (mandatory) and does so if
 *      behind(m) >= min(vmax, (len-1-x) / D): the accepted gap shrinks as
 *      the node gets closer.  Otherwise (discretionary) a side m qualifies if
 *      ahead(own) < min(v+1, vmax), ahead(m) > ahead(own), behind(m) >= vmax
 *      and m stays inside [lo, hi]; of two sides the larger ahead(m) wins,
 *      then the left one (m = l-1); it is taken if the draw u < lc_thr.
 *      Two vehicles aiming at one cell come from both sides of it; the one
 *      from the lower lane index moves, the other stays.  x and v do not
 *      change.
 *  R7  Intersections are unsignalised priority nodes.  The lead vehicle of a
 *      lane (largest x) is a candidate when len-1-x < vmax.  On its last
 *      link its trip ends at the node and it sees extra = vmax cells beyond
 *      the link end.  Otherwise it aims at lane k' = min(k, lanes'-1) of its
 *      next route link; per target lane the candidate with the smallest
 *      (rank of its link, lane) wins and sees extra = min(vmax, x_rear), the
 *      position of the rearmost vehicle of the target lane (len' if empty);
 *      every other candidate sees extra = 0.  The lead vehicle's gap is
 *      (len-1-x) + extra.  A priority vehicle within vmax cells of the node
 *      therefore blocks the minor approach: gap acceptance at the paper's
 *      5-cell interaction range.
 *  R8  A vehicle that passes the link end lands at cell x+v3-len of lane k'
 *      of the next link; exit_t[route entry of the link it left] = t.  On
 *      the last link it is removed (ARRIVED: back into parking).
 *
 * Signalised turns (same section: a virtual vehicle of maximum speed zero
 * stands at the end of the lane while the light is red):
 *  S1  A link may carry a fixed-time plan (cycle C, red R, offset O); it is
 *      red at step t iff (t + O) mod C < R, for all its lanes at once.
 *  S2  The virtual vehicle stands just beyond the last cell: while red, the
 *      lead vehicle of a lane of that link is no candidate at the node (no
 *      claim, no trip end) and sees extra = 0, so it stops by the last cell.
 *  S3  While green nothing changes: the unsignalised priority rule of R7
 *      applies among the green approaches of the node.
 *
 * Parity unpinned: the lane changes of R6 and the node arbitration of R7
 * beyond the hand-worked cases and the invariants the tests check.  The
 * paper prints no worked example or number for them, so on large networks
 * this code is held to the readings above, not to printed values.
 */
#include "transims_oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Philox-4xW-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  One round: multiply words 0 and 2 by the two  */
/* round multipliers; the new words are (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2),    */
/* hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); between rounds the key is bumped by the */
/* two Weyl constants.  Both widths come from the one template below, so    */
/* the 64-bit instance (checked against numpy's Philox) pins the structure  */
/* the 32-bit instance uses.                                                */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

#define PHILOX_4XW_10(NAME, T, MULHILO, M0, M1, W0, W1)               \
  void NAME(const T ctr[4], const T key[2], T out[4]) {               \
    T x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];             \
    T k0 = key[0], k1 = key[1];                                       \
    for (int r = 0; r < 10; ++r) {                                    \
      T hi0, lo0, hi1, lo1;                                           \
      if (r > 0) {                                                    \
        k0 = (T)(k0 + (W0));                                          \
        k1 = (T)(k1 + (W1));                                          \
      }                                                               \
      MULHILO((T)(M0), x0, &hi0, &lo0);                               \
      MULHILO((T)(M1), x2, &hi1, &lo1);                               \
      T n0 = hi1 ^ x1 ^ k0;                                           \
      T n1 = lo1;                                                     \
      T n2 = hi0 ^ x3 ^ k1;                                           \
      T n3 = lo0;                                                     \
      x0 = n0; x1 = n1; x2 = n2; x3 = n3;                             \
    }                                                                 \
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;               \
  }

PHILOX_4XW_10(orc_philox4x32_10, uint32_t, mulhilo32, 0xD2511F53u,
              0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
PHILOX_4XW_10(orc_philox4x64_10, uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull,
              0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull,
              0xBB67AE8584CAA73Bull)

/* Word 0 of Philox4x32-10 at counter (id, t, substep, 0) (reading R3). */
static uint32_t draw(uint64_t seed, int32_t id, int32_t t, uint32_t substep) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)t, substep, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[0];
}

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ---------------------------------------------------------------------- */

struct orc_sim {
  orc_params p;
  int ring;
  /* network */
  int32_t n_links;
  int32_t *len, *to, *from;
  int8_t *lanes, *rank;
  int64_t* conn_off;
  int32_t* conn_out;
  int8_t *conn_lo, *conn_hi;
  int8_t* sig;       /* signal plan of the link, -1 = none                 */
  int32_t *sig_cycle, *sig_red, *sig_off;
  int64_t* cell_off; /* lattice offset of (link, lane 0, cell 0)          */
  int64_t* lane_id;  /* global lane index of (link, lane 0)               */
  int64_t n_cells, n_lanes;
  int32_t* occ;      /* lattice: vehicle id in the cell, or -1            */
  /* vehicles */
  int32_t n;
  int32_t* depart;
  int64_t* route_off;
  int32_t* route_links;
  int32_t* exit_t;
  int8_t* status;
  int32_t *lane, *x, *v, *rptr;
  /* per-link parking FIFO: vehicles whose first link it is, by (depart,id) */
  int64_t* q_off;
  int32_t* q_ids;
  int64_t* q_head;
  /* scratch */
  int32_t *dec, *extra, *nx, *nv, *nlane, *nlink;
  int32_t *lead_x, *lead_id, *rear_x, *best;
  int32_t t;
  orc_stats st;
  int broken;
};

static int32_t cur_link(const orc_sim* s, int32_t i) {
  if (s->ring) return 0;
  return s->route_links[s->route_off[i] + s->rptr[i]];
}

static int is_last_link(const orc_sim* s, int32_t i) {
  return s->route_off[i] + s->rptr[i] + 1 == s->route_off[i + 1];
}

static int32_t* cell(orc_sim* s, int32_t link, int32_t k, int32_t c) {
  return &s->occ[s->cell_off[link] + (int64_t)k * s->len[link] + c];
}

static void* xcopy(const void* src, size_t bytes) {
  void* d = malloc(bytes ? bytes : 1);
  if (d && src && bytes) memcpy(d, src, bytes);
  if (d && !src) memset(d, 0, bytes ? bytes : 1);
  return d;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  void* ptrs[] = {s->len,     s->to,       s->from,    s->lanes,  s->rank,
                  s->conn_off, s->conn_out, s->conn_lo, s->conn_hi, s->cell_off,
                  s->lane_id, s->occ,      s->depart,  s->route_off,
                  s->route_links, s->exit_t, s->status, s->lane,  s->x,
                  s->v,       s->rptr,     s->q_off,   s->q_ids,  s->q_head,
                  s->dec,     s->extra,    s->nx,      s->nv,     s->nlane,
                  s->nlink,   s->lead_x,   s->lead_id, s->rear_x, s->best,
                  s->sig,     s->sig_cycle, s->sig_red, s->sig_off};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
  free(s);
}

#define FAIL(...)                                   \
  do {                                              \
    if (err && errlen > 0) snprintf(err, errlen, __VA_ARGS__); \
    orc_destroy(s);                                 \
    return NULL;                                    \
  } while (0)

/* sort helper for the parking FIFOs: order by (depart, id) */
static const int32_t* g_depart;
static int cmp_depart_id(const void* a, const void* b) {
  int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
  if (g_depart[i] != g_depart[j]) return g_depart[i] < g_depart[j] ? -1 : 1;
  return i < j ? -1 : (i > j);
}

orc_sim* orc_create(const orc_params* p, const orc_network* net,
                    const orc_vehicles* veh, char* err, int errlen) {
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  if (!s) return NULL;
  s->p = *p;
  s->ring = (p->flags & ORC_FLAG_RING) != 0;
  if (p->vmax < 1 || p->vmax > 7) FAIL("vmax must be 1..7");
  if (p->slow_thr > (1ull << 32) || p->lc_thr > (1ull << 32))
    FAIL("thresholds must be <= 2^32");
  if (p->lc_desp < 1) FAIL("lc_desp must be >= 1");
  int32_t L = net->n_links;
  if (L < 1) FAIL("need at least one link");
  if (s->ring && (L != 1 || net->lanes[0] != 1))
    FAIL("ring mode needs exactly one single-lane link");
  s->n_links = L;
  s->len = (int32_t*)xcopy(net->len, sizeof(int32_t) * L);
  s->to = (int32_t*)xcopy(net->to, sizeof(int32_t) * L);
  s->from = (int32_t*)xcopy(net->from, sizeof(int32_t) * L);
  s->lanes = (int8_t*)xcopy(net->lanes, L);
  s->rank = (int8_t*)xcopy(net->rank, L);
  s->cell_off = (int64_t*)xcopy(NULL, sizeof(int64_t) * (L + 1));
  s->lane_id = (int64_t*)xcopy(NULL, sizeof(int64_t) * (L + 1));
  for (int32_t l = 0; l < L; ++l) {
    if (s->lanes[l] < 1 || s->lanes[l] > 4) FAIL("link %d: lanes must be 1..4", l);
    if (s->ring) {
      if (s->len[l] < 1 || s->len[l] > 32767) FAIL("ring length out of range");
    } else {
      if (s->len[l] < p->vmax + 1 || s->len[l] > 32767)
        FAIL("link %d: length must be vmax+1..32767", l);
      if (s->from[l] == s->to[l]) FAIL("link %d is a self-loop", l);
      if (s->to[l] < 0 || s->to[l] >= net->n_nodes || s->from[l] < 0 ||
          s->from[l] >= net->n_nodes)
        FAIL("link %d: node out of range", l);
    }
    s->cell_off[l + 1] = s->cell_off[l] + (int64_t)s->lanes[l] * s->len[l];
    s->lane_id[l + 1] = s->lane_id[l] + s->lanes[l];
  }
  s->n_cells = s->cell_off[L];
  s->n_lanes = s->lane_id[L];
  if (!s->ring) {
    /* rank must be 0..127 and unique among the links that enter one node */
    uint8_t* seen = (uint8_t*)calloc((size_t)net->n_nodes * 128, 1);
    for (int32_t a = 0; a < L; ++a) {
      if (s->rank[a] < 0) {
        free(seen);
        FAIL("link %d: negative rank", a);
      }
      uint8_t* f = &seen[(size_t)s->to[a] * 128 + (size_t)s->rank[a]];
      if (*f) {
        free(seen);
        FAIL("two links enter node %d with rank %d", s->to[a], s->rank[a]);
      }
      *f = 1;
    }
    free(seen);
  }
  if (p->flags & ORC_FLAG_TURN_LANES) {
    if (!net->conn_off) FAIL("turn lanes need the lane connectivity table");
    int64_t nc = net->conn_off[L];
    s->conn_off = (int64_t*)xcopy(net->conn_off, sizeof(int64_t) * (L + 1));
    s->conn_out = (int32_t*)xcopy(net->conn_out, sizeof(int32_t) * nc);
    s->conn_lo = (int8_t*)xcopy(net->conn_lo, nc);
    s->conn_hi = (int8_t*)xcopy(net->conn_hi, nc);
  }
  /* signals (readings S1-S3) */
  s->sig = (int8_t*)xcopy(NULL, L);
  memset(s->sig, -1, L);
  if (net->signal_plan && !s->ring) {
    int32_t np = net->n_plans;
    if (np < 1 || np > 63) FAIL("1..63 signal plans");
    s->sig_cycle = (int32_t*)xcopy(net->plan_cycle, sizeof(int32_t) * np);
    s->sig_red = (int32_t*)xcopy(net->plan_red, sizeof(int32_t) * np);
    s->sig_off = (int32_t*)xcopy(net->plan_offset, sizeof(int32_t) * np);
    for (int32_t j = 0; j < np; ++j)
      if (s->sig_cycle[j] < 1 || s->sig_red[j] < 0 ||
          s->sig_red[j] > s->sig_cycle[j] || s->sig_off[j] < 0)
        FAIL("signal plan %d out of range", j);
    for (int32_t l = 0; l < L; ++l) {
      if (net->signal_plan[l] < -1 || net->signal_plan[l] >= np)
        FAIL("link %d: signal plan out of range", l);
      s->sig[l] = net->signal_plan[l];
    }
  }
  s->occ = (int32_t*)malloc(sizeof(int32_t) * (s->n_cells ? s->n_cells : 1));
  for (int64_t c = 0; c < s->n_cells; ++c) s->occ[c] = -1;

  int32_t n = veh->n;
  s->n = n;
  s->depart = (int32_t*)xcopy(veh->depart, sizeof(int32_t) * n);
  int64_t R = 0;
  if (!s->ring) {
    if (!veh->route_off) FAIL("network mode needs routes");
    R = veh->route_off[n];
    s->route_off = (int64_t*)xcopy(veh->route_off, sizeof(int64_t) * (n + 1));
    s->route_links = (int32_t*)xcopy(veh->route_links, sizeof(int32_t) * R);
    for (int32_t i = 0; i < n; ++i) {
      if (s->route_off[i + 1] <= s->route_off[i]) FAIL("vehicle %d: empty route", i);
      for (int64_t j = s->route_off[i]; j < s->route_off[i + 1]; ++j) {
        int32_t a = s->route_links[j];
        if (a < 0 || a >= L) FAIL("vehicle %d: route link out of range", i);
        if (j + 1 < s->route_off[i + 1]) {
          int32_t b = s->route_links[j + 1];
          if (b < 0 || b >= L || s->to[a] != s->from[b])
            FAIL("vehicle %d: route links %d,%d not connected", i, a, b);
          if (p->flags & ORC_FLAG_TURN_LANES) {
            int found = 0;
            for (int64_t e = s->conn_off[a]; e < s->conn_off[a + 1]; ++e)
              if (s->conn_out[e] == b) found = 1;
            if (!found) FAIL("vehicle %d: no lane connectivity %d->%d", i, a, b);
          }
        }
      }
    }
  }
  s->exit_t = (int32_t*)malloc(sizeof(int32_t) * (R ? R : 1));
  for (int64_t j = 0; j < R; ++j) s->exit_t[j] = veh->exit_t0 ? veh->exit_t0[j] : -1;
  s->status = (int8_t*)xcopy(NULL, n);
  s->lane = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->x = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->v = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->rptr = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  for (int32_t i = 0; i < n; ++i) {
    int st = veh->init_status ? veh->init_status[i] : ORC_WAITING;
    if (s->ring && st != ORC_ACTIVE) FAIL("ring mode: every vehicle starts on the ring");
    s->status[i] = (int8_t)st;
    if (st == ORC_ACTIVE) {
      int32_t rp = s->ring ? 0 : veh->init_rptr[i];
      if (!s->ring && (rp < 0 || s->route_off[i] + rp >= s->route_off[i + 1]))
        FAIL("vehicle %d: rptr out of range", i);
      s->rptr[i] = rp;
      int32_t l = cur_link(s, i);
      int32_t k = veh->init_lane[i], x = veh->init_x[i], v = veh->init_v[i];
      if (k < 0 || k >= s->lanes[l] || x < 0 || x >= s->len[l] || v < 0 ||
          v > p->vmax)
        FAIL("vehicle %d: initial placement out of range", i);
      int32_t* c = cell(s, l, k, x);
      if (*c >= 0) FAIL("vehicles %d and %d share a cell", *c, i);
      *c = i;
      s->lane[i] = k;
      s->x[i] = x;
      s->v[i] = v;
    } else if (st != ORC_WAITING && st != ORC_ARRIVED) {
      FAIL("vehicle %d: bad status", i);
    }
  }
  /* parking FIFOs */
  s->q_off = (int64_t*)xcopy(NULL, sizeof(int64_t) * (L + 1));
  s->q_ids = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->q_head = (int64_t*)xcopy(NULL, sizeof(int64_t) * L);
  if (!s->ring) {
    for (int32_t i = 0; i < n; ++i)
      if (s->status[i] == ORC_WAITING) s->q_off[s->route_links[s->route_off[i]] + 1]++;
    for (int32_t l = 0; l < L; ++l) s->q_off[l + 1] += s->q_off[l];
    int64_t* fill = (int64_t*)xcopy(s->q_off, sizeof(int64_t) * L);
    for (int32_t i = 0; i < n; ++i)
      if (s->status[i] == ORC_WAITING)
        s->q_ids[fill[s->route_links[s->route_off[i]]]++] = i;
    free(fill);
    g_depart = s->depart;
    for (int32_t l = 0; l < L; ++l) {
      qsort(s->q_ids + s->q_off[l], (size_t)(s->q_off[l + 1] - s->q_off[l]),
            sizeof(int32_t), cmp_depart_id);
      s->q_head[l] = s->q_off[l];
    }
  }
  s->dec = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->extra = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->nx = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->nv = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->nlane = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->nlink = (int32_t*)xcopy(NULL, sizeof(int32_t) * n);
  s->lead_x = (int32_t*)xcopy(NULL, sizeof(int32_t) * s->n_lanes);
  s->lead_id = (int32_t*)xcopy(NULL, sizeof(int32_t) * s->n_lanes);
  s->rear_x = (int32_t*)xcopy(NULL, sizeof(int32_t) * s->n_lanes);
  s->best = (int32_t*)xcopy(NULL, sizeof(int32_t) * s->n_lanes);
  s->t = veh->t0;
  return s;
}

/* ---------------------------------------------------------------------- */
/* Lane change helpers (reading R6), on the lattice before the sub-step.    */

static int32_t ahead(orc_sim* s, int32_t l, int32_t m, int32_t x) {
  int32_t n = 0;
  for (int32_t c = x + 1; c < s->len[l] && n < s->p.vmax; ++c) {
    if (*cell(s, l, m, c) >= 0) break;
    ++n;
  }
  return n;
}

static int32_t behind(orc_sim* s, int32_t l, int32_t m, int32_t x) {
  int32_t n = 0;
  for (int32_t c = x - 1; n < s->p.vmax; --c) {
    if (c >= 0 && *cell(s, l, m, c) >= 0) break;
    ++n; /* cells before the link start count as empty */
  }
  return n;
}

static void allowed_lanes(orc_sim* s, int32_t i, int32_t l, int32_t* lo,
                          int32_t* hi) {
  *lo = 0;
  *hi = s->lanes[l] - 1;
  if (!(s->p.flags & ORC_FLAG_TURN_LANES) || is_last_link(s, i)) return;
  int32_t next = s->route_links[s->route_off[i] + s->rptr[i] + 1];
  for (int64_t e = s->conn_off[l]; e < s->conn_off[l + 1]; ++e)
    if (s->conn_out[e] == next) {
      *lo = s->conn_lo[e];
      *hi = s->conn_hi[e];
      return;
    }
}

static int32_t decide_lane(orc_sim* s, int32_t i, int32_t t) {
  int32_t l = cur_link(s, i), k = s->lane[i], x = s->x[i], v = s->v[i];
  int32_t vmax = s->p.vmax, nl = s->lanes[l];
  int32_t lo, hi;
  allowed_lanes(s, i, l, &lo, &hi);
  if (k < lo || k > hi) { /* mandatory: one lane toward [lo, hi] */
    int32_t m = k < lo ? k + 1 : k - 1;
    int32_t need = (s->len[l] - 1 - x) / s->p.lc_desp;
    if (need > vmax) need = vmax;
    if (*cell(s, l, m, x) < 0 && behind(s, l, m, x) >= need) return m;
    return -1;
  }
  int32_t own = ahead(s, l, k, x);
  int32_t want = v + 1 < vmax ? v + 1 : vmax;
  if (own >= want) return -1;
  int32_t best = -1, best_ahead = -1;
  int32_t sides[2] = {k - 1, k + 1}; /* left side first: it wins ties */
  for (int si = 0; si < 2; ++si) {
    int32_t m = sides[si];
    if (m < 0 || m >= nl || m < lo || m > hi) continue;
    if (*cell(s, l, m, x) >= 0) continue;
    int32_t a = ahead(s, l, m, x);
    if (a <= own) continue;
    if (behind(s, l, m, x) < vmax) continue;
    if (a > best_ahead) {
      best = m;
      best_ahead = a;
    }
  }
  if (best < 0) return -1;
  if ((uint64_t)draw(s->p.seed, i, t, 0u) >= s->p.lc_thr) return -1;
  return best;
}

static void lane_change(orc_sim* s, int32_t t) {
  for (int32_t i = 0; i < s->n; ++i) {
    s->dec[i] = -1;
    if (s->status[i] != ORC_ACTIVE) continue;
    if (s->lanes[cur_link(s, i)] < 2) continue;
    s->dec[i] = decide_lane(s, i, t);
  }
  /* two vehicles aiming at one cell: the one from the lower lane moves */
  for (int32_t i = 0; i < s->n; ++i) {
    if (s->dec[i] < 0 || s->dec[i] != s->lane[i] - 1) continue;
    int32_t m = s->dec[i];
    if (m - 1 < 0) continue;
    int32_t j = *cell(s, cur_link(s, i), m - 1, s->x[i]);
    if (j >= 0 && s->dec[j] == m) s->dec[i] = -1;
  }
  /* apply all moves at once: vacate every source, then fill every target */
  for (int32_t i = 0; i < s->n; ++i)
    if (s->dec[i] >= 0) *cell(s, cur_link(s, i), s->lane[i], s->x[i]) = -1;
  for (int32_t i = 0; i < s->n; ++i)
    if (s->dec[i] >= 0) {
      int32_t* c = cell(s, cur_link(s, i), s->dec[i], s->x[i]);
      if (*c >= 0) s->broken = 1;
      *c = i;
      s->lane[i] = s->dec[i];
      s->st.lane_changes++;
    }
}

/* ---------------------------------------------------------------------- */

static void account_lanes(orc_sim* s) {
  /* lead (largest x) and rear (smallest x) of every lane, from the vehicles */
  for (int64_t q = 0; q < s->n_lanes; ++q) {
    s->lead_x[q] = -1;
    s->lead_id[q] = -1;
    s->rear_x[q] = -1;
  }
  for (int32_t i = 0; i < s->n; ++i) {
    if (s->status[i] != ORC_ACTIVE) continue;
    int64_t q = s->lane_id[cur_link(s, i)] + s->lane[i];
    if (s->x[i] > s->lead_x[q]) {
      s->lead_x[q] = s->x[i];
      s->lead_id[q] = i;
    }
    if (s->rear_x[q] < 0 || s->x[i] < s->rear_x[q]) s->rear_x[q] = s->x[i];
  }
  for (int32_t l = 0; l < s->n_links; ++l)
    for (int32_t k = 0; k < s->lanes[l]; ++k) {
      int64_t q = s->lane_id[l] + k;
      if (s->lead_id[q] >= 0) s->st.c_occ += s->len[l];
      else s->rear_x[q] = s->len[l];
    }
}

/* Reading S1: is the light at the end of link l red in step t? */
static int is_red(const orc_sim* s, int32_t l, int32_t t) {
  int8_t j = s->sig[l];
  if (j < 0) return 0;
  return (int32_t)(((int64_t)t + s->sig_off[j]) % s->sig_cycle[j]) < s->sig_red[j];
}

/* Readings R7, S2, S3. */
static void arbitrate(orc_sim* s) {
  int32_t vmax = s->p.vmax;
  for (int32_t i = 0; i < s->n; ++i) s->extra[i] = 0;
  for (int64_t q = 0; q < s->n_lanes; ++q) s->best[q] = 1 << 30;
  for (int pass = 0; pass < 2; ++pass) {
    for (int32_t l = 0; l < s->n_links; ++l)
      for (int32_t k = 0; k < s->lanes[l]; ++k) {
        int32_t i = s->lead_id[s->lane_id[l] + k];
        if (i < 0 || s->len[l] - 1 - s->x[i] >= vmax) continue;
        if (is_red(s, l, s->t)) continue; /* S2: the virtual vehicle */
        if (is_last_link(s, i)) {
          s->extra[i] = vmax;
          continue;
        }
        int32_t nl = s->route_links[s->route_off[i] + s->rptr[i] + 1];
        int32_t nk = k < s->lanes[nl] - 1 ? k : s->lanes[nl] - 1;
        int64_t tq = s->lane_id[nl] + nk;
        int32_t key = s->rank[l] * 8 + k;
        if (pass == 0) {
          if (key < s->best[tq]) s->best[tq] = key;
        } else if (key == s->best[tq]) {
          s->extra[i] = s->rear_x[tq] < vmax ? s->rear_x[tq] : vmax;
        }
      }
  }
}

static void network_step(orc_sim* s) {
  int32_t t = s->t, vmax = s->p.vmax;
  /* 1. leave parking (reading R5) */
  for (int32_t l = 0; l < s->n_links; ++l) {
    if (s->q_head[l] >= s->q_off[l + 1]) continue;
    int32_t i = s->q_ids[s->q_head[l]];
    if (s->depart[i] > t) continue;
    for (int32_t k = 0; k < s->lanes[l]; ++k) {
      int32_t* c = cell(s, l, k, 0);
      if (*c >= 0) continue;
      *c = i;
      s->status[i] = ORC_ACTIVE;
      s->lane[i] = k;
      s->x[i] = 0;
      s->v[i] = 0;
      s->rptr[i] = 0;
      s->q_head[l]++;
      s->st.insertions++;
      break;
    }
  }
  /* 2. first sub-step: lane changes (reading R6) */
  if (s->p.flags & ORC_FLAG_LANE_CHANGE) lane_change(s, t);
  /* 3. intersections (reading R7) */
  account_lanes(s);
  arbitrate(s);
  /* 4. second sub-step: speeds from the lattice as it is now, then move */
  for (int32_t i = 0; i < s->n; ++i) {
    if (s->status[i] != ORC_ACTIVE) continue;
    int32_t l = cur_link(s, i), k = s->lane[i], x = s->x[i];
    int32_t gap = -1;
    /* empty cells to the vehicle ahead; since v1 <= vmax only min(gap, vmax)
       matters, so the scan stops after vmax cells */
    int32_t c;
    for (c = x + 1; c < s->len[l] && c <= x + vmax; ++c)
      if (*cell(s, l, k, c) >= 0) {
        gap = c - x - 1;
        break;
      }
    if (gap < 0) gap = (c > x + vmax) ? vmax : (s->len[l] - 1 - x) + s->extra[i];
    int32_t v1 = s->v[i] + 1 < vmax ? s->v[i] + 1 : vmax;
    int32_t v2 = v1 < gap ? v1 : gap;
    int32_t v3 = v2;
    if (v2 > 0 && (uint64_t)draw(s->p.seed, i, t, 1u) < s->p.slow_thr) v3 = v2 - 1;
    s->nv[i] = v3;
    s->nx[i] = x + v3;
    s->nlink[i] = l;
    s->nlane[i] = k;
    s->st.veh_updates++;
    s->st.sum_v += v3;
  }
  for (int32_t i = 0; i < s->n; ++i)
    if (s->status[i] == ORC_ACTIVE) *cell(s, cur_link(s, i), s->lane[i], s->x[i]) = -1;
  for (int32_t i = 0; i < s->n; ++i) {
    if (s->status[i] != ORC_ACTIVE) continue;
    int32_t l = s->nlink[i], k = s->nlane[i], x = s->nx[i];
    s->v[i] = s->nv[i];
    if (x >= s->len[l]) { /* reading R8 */
      s->exit_t[s->route_off[i] + s->rptr[i]] = t;
      if (is_last_link(s, i)) {
        s->status[i] = ORC_ARRIVED;
        s->st.exits++;
        continue;
      }
      x -= s->len[l];
      s->rptr[i]++;
      l = cur_link(s, i);
      k = k < s->lanes[l] - 1 ? k : s->lanes[l] - 1;
      s->st.crossings++;
    }
    int32_t* c = cell(s, l, k, x);
    if (*c >= 0) s->broken = 1; /* two vehicles in one cell */
    *c = i;
    s->lane[i] = k;
    s->x[i] = x;
  }
}

/* Reading R4. */
static void ring_step(orc_sim* s) {
  int32_t t = s->t, vmax = s->p.vmax, L = s->len[0];
  s->st.c_occ += s->n > 0 ? L : 0;
  for (int32_t i = 0; i < s->n; ++i) {
    int32_t x = s->x[i];
    /* empty cells to the next vehicle around the ring, capped at vmax (the
       lone vehicle sees L-1) */
    int32_t lim = vmax < L - 1 ? vmax : L - 1;
    int32_t gap = lim;
    for (int32_t d = 1; d <= lim; ++d)
      if (s->occ[(x + d) % L] >= 0) {
        gap = d - 1;
        break;
      }
    int32_t v1 = s->v[i] + 1 < vmax ? s->v[i] + 1 : vmax;
    int32_t v2 = v1 < gap ? v1 : gap;
    int32_t v3 = v2;
    if (v2 > 0 && (uint64_t)draw(s->p.seed, i, t, 1u) < s->p.slow_thr) v3 = v2 - 1;
    s->nv[i] = v3;
    s->nx[i] = (x + v3) % L;
    s->st.veh_updates++;
    s->st.sum_v += v3;
  }
  for (int32_t i = 0; i < s->n; ++i) s->occ[s->x[i]] = -1;
  for (int32_t i = 0; i < s->n; ++i) {
    if (s->occ[s->nx[i]] >= 0) s->broken = 1;
    s->occ[s->nx[i]] = i;
    s->x[i] = s->nx[i];
    s->v[i] = s->nv[i];
  }
}

int orc_step(orc_sim* s, int32_t n) {
  for (int32_t k = 0; k < n; ++k) {
    if (s->ring) ring_step(s);
    else network_step(s);
    s->t++;
  }
  return s->broken ? -1 : 0;
}

void orc_get_state(const orc_sim* s, int8_t* status, int32_t* link,
                   int8_t* lane, int32_t* x, int8_t* v, int32_t* rptr,
                   int32_t* exit_t) {
  for (int32_t i = 0; i < s->n; ++i) {
    int act = s->status[i] == ORC_ACTIVE;
    if (status) status[i] = s->status[i];
    if (link) link[i] = act ? cur_link(s, i) : -1;
    if (lane) lane[i] = act ? (int8_t)s->lane[i] : 0;
    if (x) x[i] = act ? s->x[i] : 0;
    if (v) v[i] = act ? (int8_t)s->v[i] : 0;
    if (rptr) rptr[i] = act ? s->rptr[i] : 0;
  }
  if (exit_t && !s->ring)
    memcpy(exit_t, s->exit_t, sizeof(int32_t) * (size_t)s->route_off[s->n]);
}

/* State hash: sum over vehicles of a SplitMix64 mix of (id, status, and for
   active vehicles link, lane, x, v, rptr), modulo 2^64. */
static uint64_t vehicle_hash(int32_t id, int st, int32_t link, int32_t lane,
                             int32_t x, int32_t v, int32_t rptr) {
  uint64_t w = (uint64_t)st | ((uint64_t)(uint32_t)lane << 4) |
               ((uint64_t)(uint32_t)v << 8) |
               ((uint64_t)((uint32_t)x & 0xFFFFu) << 16) |
               ((uint64_t)(uint32_t)link << 32);
  uint64_t h = orc_mix64(orc_mix64((uint64_t)(uint32_t)id) ^ w);
  return orc_mix64(h ^ (uint64_t)(uint32_t)rptr);
}

void orc_get_stats(const orc_sim* s, orc_stats* out) {
  *out = s->st;
  out->t = s->t;
  out->n_waiting = out->n_active = out->n_arrived = 0;
  uint64_t h = 0;
  for (int32_t i = 0; i < s->n; ++i) {
    int st = s->status[i];
    if (st == ORC_WAITING) out->n_waiting++;
    if (st == ORC_ARRIVED) out->n_arrived++;
    if (st == ORC_ACTIVE) {
      out->n_active++;
      h += vehicle_hash(i, st, cur_link(s, i), s->lane[i], s->x[i], s->v[i],
                        s->rptr[i]);
    } else {
      h += vehicle_hash(i, st, 0, 0, 0, 0, 0);
    }
  }
  out->hash = h;
}
