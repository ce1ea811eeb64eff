// tiler.h -- assignment of links to workgroup tiles.
//
// The paper decomposes the street network into domains of similar load by
// orthogonal recursive bisection (Section "Graph partitioning": nodes weighted
// by the load of their links, cuts alternating between the two axes,
// recursion on both halves) and measures the result by the partition
// efficiency e_dmn = (load of the optimal partition) / (load of the largest
// partition).  On one GPU the same ideas order the links so that a tile (one
// wavefront's worth of whole links) and an XCD's share of tiles are
// geographically compact, which keeps a node's incoming and outgoing links
// -- the only cross-tile traffic -- close together.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "transims.h"

namespace tr {

// Reorders `order` (link ids) by ORB over the link midpoints (mx, my) with
// weights w: each range is cut at its weighted median along x, then y, ...
void orb_order(std::vector<int32_t>& order, const std::vector<double>& mx,
               const std::vector<double>& my, const std::vector<double>& w);

// Packs consecutive links (lanes[l] lanes each) into tiles of at most
// tile_lanes lanes; a tile never splits a link.  Returns {first lane, lanes}.
std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes, int tile_lanes);
// The same, and a tile also takes no link that would bring it past max_cells
// cells (len x lanes), unless the tile is still empty.
std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes,
                             const std::vector<int32_t>& len, int tile_lanes,
                             int64_t max_cells);

// The same with a weight per link (the measured cost of adaptive load
// balancing): a tile also takes no link that would bring its weight past
// max_weight, unless the tile is still empty.
std::vector<int2> pack_tiles(const std::vector<int32_t>& lanes,
                             const std::vector<int32_t>& len,
                             const std::vector<double>& weight, int tile_lanes,
                             int64_t max_cells, double max_weight);

// Deals a list of tiles to `domains` XCDs: XCD x gets the x-th contiguous
// chunk, and position p of the result runs on XCD p mod domains.
std::vector<int2> xcd_interleave(const std::vector<int2>& tiles, int domains);

// e_dmn over the 8 XCD domains and mean/max over tiles, from link weights.
sim_tiling tiling_metrics(const std::vector<int2>& tiles,
                          const std::vector<int32_t>& lanes,
                          const std::vector<int32_t>& lane0,
                          const std::vector<double>& weight);

}  // namespace tr
