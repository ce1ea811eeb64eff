// tiler.cpp -- ORB ordering of links, tile packing, XCD dealing, e_dmn.
#include "tiler.h"

#include <algorithm>
#include <numeric>

namespace tr {

namespace {

void orb_rec(std::vector<int32_t>& o, int64_t lo, int64_t hi, int depth,
             const std::vector<double>& mx, const std::vector<double>& my,
             const std::vector<double>& w) {
  if (hi - lo <= 4) return;
  const std::vector<double>* ax = (depth & 1) ? &my : &mx;
  double a0 = (*ax)[o[lo]], a1 = a0;
  for (int64_t i = lo; i < hi; ++i) {
    a0 = std::min(a0, (*ax)[o[i]]);
    a1 = std::max(a1, (*ax)[o[i]]);
  }
  if (a0 == a1) ax = (depth & 1) ? &mx : &my;  // degenerate along this axis
  std::stable_sort(o.begin() + lo, o.begin() + hi, [&](int32_t a, int32_t b) {
    const double pa = (*ax)[a], pb = (*ax)[b];
    return pa < pb || (pa == pb && a < b);
  });
  double total = 0;
  for (int64_t i = lo; i < hi; ++i) total += w[o[i]];
  double acc = 0;
  int64_t cut = lo + (hi - lo) / 2;
  if (total > 0) {
    for (int64_t i = lo; i < hi; ++i) {
      acc += w[o[i]];
      if (acc >= 0.5 * total) {
        cut = i + 1;
        break;
      }
    }
  }
  cut = std::min(std::max(cut, lo + 1), hi - 1);
  orb_rec(o, lo, cut, depth + 1, mx, my, w);
  orb_rec(o, cut, hi, depth + 1, mx, my, w);
}

}  // namespace

void orb_order(std::vector<int32_t>& order, const std::vector<double>& mx,
               const std::vector<double>& my, const std::vector<double>& w) {
  orb_rec(order, 0, (int64_t)order.size(), 0, mx, my, w);
}

std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes, int tile_lanes) {
  std::vector<int2> tiles;
  int32_t first = 0, cur = 0;
  for (size_t l = 0; l < lanes.size(); ++l) {
    if (cur > 0 && cur + lanes[l] > tile_lanes) {
      tiles.push_back(make_int2(first, cur));
      first += cur;
      cur = 0;
    }
    cur += lanes[l];
  }
  if (cur > 0) tiles.push_back(make_int2(first, cur));
  return tiles;
}

std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes,
                             const std::vector<int32_t>& len, int tile_lanes,
                             int64_t max_cells) {
  std::vector<int2> tiles;
  int32_t first = 0, cur = 0;
  int64_t cells = 0;
  for (size_t l = 0; l < lanes.size(); ++l) {
    const int64_t c = (int64_t)lanes[l] * len[l];
    if (cur > 0 && (cur + lanes[l] > tile_lanes || cells + c > max_cells)) {
      tiles.push_back(make_int2(first, cur));
      first += cur;
      cur = 0;
      cells = 0;
    }
    cur += lanes[l];
    cells += c;
  }
  if (cur > 0) tiles.push_back(make_int2(first, cur));
  return tiles;
}

std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes,
                             const std::vector<int32_t>& len,
                             const std::vector<double>& weight, int tile_lanes,
                             int64_t max_cells, double max_weight) {
  std::vector<int2> tiles;
  int32_t first = 0, cur = 0;
  int64_t cells = 0;
  double wsum = 0.0;
  for (size_t l = 0; l < lanes.size(); ++l) {
    const int64_t c = (int64_t)lanes[l] * len[l];
    if (cur > 0 && (cur + lanes[l] > tile_lanes || cells + c > max_cells ||
                    wsum + weight[l] > max_weight)) {
      tiles.push_back(make_int2(first, cur));
      first += cur;
      cur = 0;
      cells = 0;
      wsum = 0.0;
    }
    cur += lanes[l];
    cells += c;
    wsum += weight[l];
  }
  if (cur > 0) tiles.push_back(make_int2(first, cur));
  return tiles;
}

std::vector<int2> xcd_interleave(const std::vector<int2>& tiles, int domains) {
  const int64_t n = (int64_t)tiles.size();
  // the first n mod domains chunks hold one tile more, so that the last,
  // partial round of positions is exactly those chunks' XCDs
  const int64_t q = n / domains, rem = n % domains;
  std::vector<int64_t> start(domains + 1);
  for (int x = 0; x <= domains; ++x) start[x] = q * x + std::min<int64_t>(x, rem);
  std::vector<int2> out;
  out.reserve(n);
  for (int64_t r = 0;; ++r) {
    bool any = false;
    for (int x = 0; x < domains; ++x)
      if (start[x] + r < start[x + 1]) {
        out.push_back(tiles[start[x] + r]);
        any = true;
      }
    if (!any) break;
  }
  return out;
}

sim_tiling tiling_metrics(const std::vector<int2>& tiles,
                          const std::vector<int32_t>& lanes,
                          const std::vector<int32_t>& lane0,
                          const std::vector<double>& weight) {
  sim_tiling m{};
  m.n_tiles = (int32_t)tiles.size();
  std::vector<double> tw(tiles.size(), 0.0);
  size_t l = 0;
  for (size_t t = 0; t < tiles.size(); ++t) {
    while (l < lanes.size() && lane0[l] < tiles[t].x + tiles[t].y) {
      tw[t] += weight[l];
      ++l;
    }
  }
  const double sum = std::accumulate(tw.begin(), tw.end(), 0.0);
  const double mx = tw.empty() ? 0 : *std::max_element(tw.begin(), tw.end());
  m.e_tile = mx > 0 ? sum / tw.size() / mx : 1.0;
  // position p of the dealt list runs on XCD p mod 8
  std::vector<int2> idx(tiles.size());
  for (size_t t = 0; t < tiles.size(); ++t) idx[t] = make_int2((int)t, 0);
  const std::vector<int2> dealt = xcd_interleave(idx, 8);
  double dom[8] = {0};
  for (size_t p = 0; p < dealt.size(); ++p) dom[p % 8] += tw[dealt[p].x];
  const double dmax = *std::max_element(dom, dom + 8);
  m.e_dmn = dmax > 0 ? sum / 8 / dmax : 1.0;
  return m;
}

}  // namespace tr
