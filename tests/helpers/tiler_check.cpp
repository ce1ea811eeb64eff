// Drives the library's host tiling code (csrc/tiler.cpp) for the tiling
// tests: reads a case from stdin, prints the result as whitespace-separated
// integers.
//   pack  T C W n  lanes[n] len[n] weight[n]  -> pairs (first lane, lanes)
//         (C < 0: no cell cap; W < 0: no weight cap)
//   deal  n  -> for each position, the input index dealt there (8 XCDs)
//   orb   n  x[n] y[n] w[n]  -> the ORB order of the n points
#include <cstdio>
#include <cstring>
#include <vector>

#include "tiler.h"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  if (!std::strcmp(argv[1], "pack")) {
    int T, n;
    long long C;
    double W;
    if (std::scanf("%d %lld %lf %d", &T, &C, &W, &n) != 4) return 3;
    std::vector<int32_t> lanes(n), len(n);
    std::vector<double> w(n);
    for (auto& v : lanes) std::scanf("%d", &v);
    for (auto& v : len) std::scanf("%d", &v);
    for (auto& v : w) std::scanf("%lf", &v);
    std::vector<int2> t;
    if (C < 0 && W < 0) t = tr::pack_tiles(lanes, T);
    else if (W < 0) t = tr::pack_tiles(lanes, len, T, C);
    else t = tr::pack_tiles(lanes, len, w, T, C < 0 ? (1LL << 62) : C, W);
    for (const int2& x : t) std::printf("%d %d\n", x.x, x.y);
  } else if (!std::strcmp(argv[1], "deal")) {
    int n;
    if (std::scanf("%d", &n) != 1) return 3;
    std::vector<int2> in(n);
    for (int i = 0; i < n; ++i) in[i] = make_int2(i, 0);
    for (const int2& x : tr::xcd_interleave(in, 8)) std::printf("%d\n", x.x);
  } else if (!std::strcmp(argv[1], "orb")) {
    int n;
    if (std::scanf("%d", &n) != 1) return 3;
    std::vector<double> x(n), y(n), w(n);
    for (auto& v : x) std::scanf("%lf", &v);
    for (auto& v : y) std::scanf("%lf", &v);
    for (auto& v : w) std::scanf("%lf", &v);
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    tr::orb_order(order, x, y, w);
    for (int32_t v : order) std::printf("%d\n", v);
  } else {
    return 2;
  }
  return 0;
}
