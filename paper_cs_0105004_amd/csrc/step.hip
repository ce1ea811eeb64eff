// step.hip -- the one-kernel form of the TRANSIMS per-second update
// (gfx950), used for scenarios without lane changes whose links all have at
// least 2*vmax cells: one wavefront per tile performs the whole step, with
// the state kept by step parity so that no tile overwrites what another may
// still read.
#include "device.h"
#include "kernels.h"
#include "philox.h"
#include "transims.h"

namespace tr {

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
// Addresses only a vehicle crossing a node uses.  They wait in LDS, which
// keeps them out of the scalar registers through the move.
struct CrossPtrs {
  const uint32_t* route_info;
  int32_t* exit_t;
  unsigned long long* arr_out;  // arrival bits written this step
};

__device__ __forceinline__ void step_load(
    StepGroup& G, int g0, int i, int total, int nl, int vp,
    const int* s_pre, const int* s_len, const int* s_base, const int* s_hp,
    GAS v2u* hot, GAS uint32_t* hot_w, GAS v2i* cold) {
#pragma unroll
  for (int c = 0; c < kGroup; ++c) {
    const int fr0 = (g0 + c) * kWave, fr = fr0 + i;
    const int f = max(min(fr, total - 1), 0);
    const int lo = wave_lane_of(vp, nl, max(min(fr0, total - 1), 0),
                                max(min(fr0 + kWave - 1, total - 1), 0), f);
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
    GAS v2i* cold, const CrossPtrs* s_xp, GAS v4i* __restrict__ ha_out,
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
      } else if (nw != hw.x) {  // a vehicle that stays put keeps its word
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
      const CrossPtrs xp = *s_xp;
      gp(xp.exit_t)[rp] = cx.t;
      s_left[li] = 1;
      if (fl & kFlLast) {
        ++exits;
      } else {
        const uint32_t nfl = rinfo_flags((uint32_t)cw.y);
        const int tg = s_tgt[li];
        hb_out[tg] = (nfl & kFlLast) ? 0 : (int)gp(xp.route_info)[rp + 2];
        ha_out[tg] = (v4i){cx.t, (int)pack_xvf(nx - llen, v3, nfl),
                           (int)hw.y, rp + 1};
        ht_out[tg] = (cx.t << 1) | (nx == llen ? 1 : 0);
        atomicOr(&xp.arr_out[tg >> 6], 1ull << (tg & 63));
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
template <bool kBatched, bool kSkip>
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
  __shared__ CrossPtrs s_xp;
  __shared__ int s_wake;  // the tile's wake step (kSkip)
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
  const int i = threadIdx.x;
  const int nl = w.z;
  const bool act = i < nl;
  const int g = w.y + i;

  // 0. which lanes have anything to do (kSkip): those that held a vehicle
  // at the start of this step or of the one before (the tile's mask), those
  // a vehicle was handed over into (the arrival bits), and every lane when
  // a parking-queue head of the tile may leave (the tile's wake step).  A
  // lane outside these is empty and stays empty, and both of its parity
  // buffers already hold that state, so it is neither read nor written.
  // Without kSkip every lane is looked at; both forms keep the masks, wake
  // steps and arrival bits up to date, so that either may follow the other.
  const long long nft = S.n_ftiles;
  unsigned long long* arr_in = S.arr_bits + (p ^ 1) * ((Q + 63) >> 6);
  if (threadIdx.x == 0)
    s_xp = CrossPtrs{S.route_info, S.exit_t, S.arr_bits + p * ((Q + 63) >> 6)};
  bool full = true, arrb = false, live = act;
  if (kSkip) {
    const unsigned long long own = S.tile_live[p * nft + w.w];
    const int wake = S.tile_wake[p * nft + w.w];
    if (threadIdx.x == 0) s_wake = wake;
    full = wake <= t;
    arrb = act && ((arr_in[(act ? g : w.y) >> 6] >> (g & 63)) & 1ull) != 0;
    live = act && (full || ((own >> i) & 1ull) != 0 || arrb);
  }
  // 1. what every live lane needs from the previous step, in one round:
  // its static word, its state, the tag of the last handoff into it and the
  // departure time of its link's queue head
  v2i bm = {0, 0};
  v4i st = {0, 0, 0, 0};
  int htag = kTagNone, qn = INT32_MAX;
  if (kSkip) {
    if (live) {
      bm = lane_bm[g];
      st = ls_cur[g];
      qn = qn_cur[g];
      if (arrb) htag = ht_in[g];
    }
  } else {
    // (threads past the tile's lanes read its first lane and drop it, so
    // that no load waits behind a branch)
    const int gg = act ? g : w.y;
    bm = lane_bm[gg];
    st = ls_cur[gg];
    htag = ht_in[gg];
    qn = qn_cur[gg];
    if (!act) {
      bm = (v2i){0, 0};
      st = (v4i){0, 0, 0, 0};
      htag = kTagNone;
      qn = INT32_MAX;
    }
  }
  load_plans(S, s_plans);
  const uint32_t meta = (uint32_t)bm.y;
  // (links of a one-kernel slot have at least 2 vmax cells, so len > 1
  // marks a live lane from here on)
  const int len = live ? lmeta_len(meta) : 1;
  const int k = lmeta_k(meta), lanes = lmeta_lanes(meta);
  const int key = lmeta_rank(meta) * 8 + k;
  const int head = hc_head(st.w);
  const int cnt = live ? hc_cnt(st.w) : 0;
  const uint32_t lead_w = (uint32_t)st.x;
  // a vehicle handed over in the previous step joins at the rear (its
  // record is read below); the tag says whether it landed on cell 0
  bool arr = false;
  if (live && (htag >> 1) == t - 1) {
    if (cnt >= len) atomicOr(S.err, SIM_DEVERR_LANE_FULL);
    else arr = true;
  }
  // the arrival bit is consumed: this parity's bits are set again by the
  // handoffs of the next step but one
  if (arr) atomicAnd(&arr_in[g >> 6], ~(1ull << (g & 63)));
  const int rear_x =
      arr ? ((htag & 1) ? 0 : 1) : (cnt > 0 ? xvf_x((uint32_t)st.z) : 1);
  const bool empty0 = len > 1 && rear_x != 0;
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
  const bool cand = cnt > 0 && len - 1 - xvf_x(lead_w) < vmax &&
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
  if (act) {  // (a lane that is not live holds no vehicle)
    s_base[i] = bm.x;
    s_hp[i] = hc_make(head, 0, 0);
    s_len[i] = len;
    s_cnt0[i] = cnt;
    s_tgt[i] = tgt;
    s_left[i] = 0;
    s_ends[i] = make_int4(0, 0, 0, 0);
  }
  const int cntn = cnt + n_new;
  const int incl = wave_scan(cntn);
  const int total = wave_last(incl);  // in a scalar register
  if (i < nl) s_pre[i] = incl - cntn;
  if (i == 0) s_pre[nl] = total;
  const unsigned long long cocc =
      wave_sum(cntn > 0 ? len : 0);
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
    step_load(G, gr, i, total, nl, incl - cntn, s_pre, s_len, s_base, s_hp,
              hot, hot_w, cold);
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
      if (len > 1) {
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
             s_ends, s_second, s_left, hot, hot_w, cold, &s_xp, ha_out,
             hb_out, ht_out, sumv, cross, exits);
  }
  wave_lds_sync();

  // 4. the lanes for the next step, and the claims of their new leads;
  // with them the tile's control words for the next step: the lanes that
  // hold a vehicle now or did at its start, and the wake step -- unchanged
  // unless this step looked at every lane, which gives the earliest
  // departure of a queue head (or the next step itself if a queue moved
  // on, so that the next step copies the new head's departure into the
  // other parity buffer)
  bool held = false;
  int qnx = INT32_MAX;
  if (len > 1) {
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
    held = c1 > 0 || s_cnt0[i] > 0;
    if (c1 > 0 && len - 1 - xvf_x((uint32_t)e.x) < vmax &&
        !(xvf_fl((uint32_t)e.x) & kFlLast) && !sig_red(s_plans, meta, t + 1)) {
      const uint32_t ni = (uint32_t)e.y;
      atomicMin((int*)&cl_nxt[rinfo_lane0(ni) + min(k, rinfo_lanes(ni) - 1)],
                key);
    }
    if (k == 0) {
      qnx = qn;
      if (link_ins) {
        lane_qhead[g] = qh + 1;
        lane_qrec[g] = nrec;
        qnx = qh + 1 < qend ? (nrec.y & ((1 << kDepartBits) - 1)) : INT32_MAX;
      }
      qn_nxt[g] = qnx;
    }
  }
  const unsigned long long own1 = __ballot(held);
  sumv = wave_sum((int)sumv);
  cross = wave_sum((int)cross);
  exits = wave_sum((int)exits);
  const unsigned long long n_ins = wave_sum(ins);
  int wake1;
  if (kSkip && s_wake > t) {
    wake1 = s_wake;
  } else {
    qnx = wave_min(qnx);
    wake1 = n_ins ? min(qnx, t + 1) : qnx;
  }
  if (i == 0) {
    S.tile_live[(p ^ 1) * nft + w.w] = own1;
    S.tile_wake[(p ^ 1) * nft + w.w] = wake1;
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

// ---- launchers -------------------------------------------------------------

hipError_t launch_step(const DevScen* d_descs, int slot, const int4* d_work,
                       int n_work, int step, bool skip, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  (void)hipGetLastError();
  const dim3 grid(n_work), block(kWave);
  if (slot < 0) {
    if (skip)
      hipLaunchKernelGGL((k_step<true, true>), grid, block, 0, s, d_descs, 0,
                         d_work, step);
    else
      hipLaunchKernelGGL((k_step<true, false>), grid, block, 0, s, d_descs, 0,
                         d_work, step);
  } else {
    if (skip)
      hipLaunchKernelGGL((k_step<false, true>), grid, block, 0, s, d_descs,
                         slot, d_work, step);
    else
      hipLaunchKernelGGL((k_step<false, false>), grid, block, 0, s, d_descs,
                         slot, d_work, step);
  }
  return hipGetLastError();
}

void* step_kernel(bool batched, bool skip) {
  if (batched)
    return skip ? reinterpret_cast<void*>(&k_step<true, true>)
                : reinterpret_cast<void*>(&k_step<true, false>);
  return skip ? reinterpret_cast<void*>(&k_step<false, true>)
              : reinterpret_cast<void*>(&k_step<false, false>);
}

}  // namespace tr
