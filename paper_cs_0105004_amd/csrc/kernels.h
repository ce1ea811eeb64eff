// kernels.h -- launchers of the libtransims device kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

namespace tr {

// One step of every tile in `work` ({slot, first lane, lanes, tile}, in
// dispatch order; slot >= 0: every item belongs to that slot):
// the front kernel merges arrivals, lets vehicles leave parking, runs the
// lane-change sub-step and publishes per-lane summaries; the back kernel
// resolves the intersections and moves every vehicle (second sub-step).
// lc_words: most lattice words of a tile's lane-changing links (each lane
// ceil(len/32) words); the lane-change sub-step takes kLcBytesPerWord bytes
// of LDS per word.
// pieces: most move wavefronts per tile (single slot; 1 = one per tile)
hipError_t launch_front(const DevScen* d_descs, int slot, const int4* d_work,
                        int n_work, int pieces, int step, int lc_words,
                        hipStream_t s);
// The move kernel: one wavefront per work item plus, for a single slot,
// n_extra wavefronts for the runs of heavy tiles the front kernel listed.
hipError_t launch_back(const DevScen* d_descs, int slot, const int4* d_work,
                       int n_work, int n_extra, int step, hipStream_t s);
// One kernel for the whole step, for slots whose state is kept by step
// parity (DevScen::fused); work items as above, one wavefront each.  With
// skip, lanes that are empty and stay empty are neither read nor written
// (worth it when many more tiles than fit on the device at once share the
// launch); results are the same either way.
hipError_t launch_step(const DevScen* d_descs, int slot, const int4* d_work,
                       int n_work, int step, bool skip, hipStream_t s);
// Host stubs of the step kernels, for building HIP graphs:
//   step(descs, slot, work, step) (step_kernel(batched, skip)),
//   front(descs, slot, work, pieces, step), back(descs, slot, work, n_work,
//   step), advance(descs, slots, n, k)
void* step_kernel(bool batched, bool skip);
void* front_kernel(bool batched);
void* back_kernel(bool batched);
void* advance_kernel();
// order(descs, work, n, snap): each XCD's positions of the two-kernel
// work list of n items, the tile that took longest in the front kernel
// since the last ordering first; snap[n] holds each position's cycle count
// at the last ordering.  One workgroup of kOrderThreads per XCD, for at
// most kOrderMax positions per XCD (8 * kOrderMax items).
void* order_kernel();
constexpr int kOrderThreads = 1024, kOrderMax = 2048;
constexpr int kFrontThreads = kWave, kBackThreadsPerPiece = kWave;
constexpr int kLcBytesPerWord = 14;
// A link has at most 4 lanes of at most 32767 cells (1024 words each), and a
// tile of lane-changing links with more than one link holds at most
// tile_cells <= 65536 cells, so no tile needs more words than this.
constexpr int kMaxLcWords = 4096;
// descs[slots[i]].t += k for i < n
hipError_t launch_advance(DevScen* d_descs, const int* d_slots, int n, int k,
                          hipStream_t s);
// All n_steps of each listed ring slot in one launch (one workgroup each).
hipError_t launch_ring(DevScen* d_descs, const int* d_slots, int n,
                       int n_steps, hipStream_t s);
// out[0..C_N) counter sums, out[C_N] active, out[C_N+1] hash,
// out[C_N+2] waiting; out must be zeroed first.
hipError_t launch_stats(const DevScen* d_desc, unsigned long long* d_out,
                        int ring, hipStream_t s);

// The device scratch of sim_step_noalloc (csrc/scratch.hip): at most
// kScratchWork work items and kScratchSlots listed slots per call.
constexpr int kScratchWork = 1 << 17;
constexpr int kScratchSlots = 1 << 14;
// Looks up the scratch's address on `device`, which must be current; once
// per device, later calls return at once.
hipError_t scratch_init(int device);
// The scratch's device address on `device` (nullptr before scratch_init).
void* scratch_ptr(int device);

struct ExportBufs {
  int8_t* status;
  int32_t* link;
  int8_t* lane;
  int32_t* x;
  int8_t* v;
  int32_t* rptr;
};
hipError_t launch_export(const DevScen* d_desc, ExportBufs out, int n_veh,
                         int n_links, int n_lanes, int ring, hipStream_t s);

}  // namespace tr
