// hip_stub.cpp -- a stand-in for the HIP runtime and for libtransims'
// kernel launchers, for testing the library's host code on a machine
// without a GPU.  Test infrastructure only: linked with transims.cpp and
// tiler.cpp into a separate host-only library by tests/test_host_logic.py.
//
// "Device" memory is host memory, copies and fills are memcpy and memset,
// and every kernel launch does nothing.  Nothing here computes a step: the
// harness exercises argument checks, slot bookkeeping, tiling, workspace
// carving and the uploads of sim_load_network / sim_load_vehicles, and the
// copies back of sim_read_state.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "kernels.h"

extern "C" {

hipError_t hipGetDevice(int* deviceId) {
  *deviceId = 0;
  return hipSuccess;
}

hipError_t hipSetDevice(int deviceId) {
  return deviceId == 0 ? hipSuccess : hipErrorInvalidDevice;
}

hipError_t hipMalloc(void** ptr, size_t size) {
  *ptr = std::aligned_alloc(256, (size + 255) / 256 * 256);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void* ptr) {
  std::free(ptr);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t sizeBytes,
                          hipMemcpyKind, hipStream_t) {
  if (sizeBytes) std::memmove(dst, src, sizeBytes);
  return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int value, size_t sizeBytes, hipStream_t) {
  if (sizeBytes) std::memset(dst, value, sizeBytes);
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

const char* hipGetErrorString(hipError_t) { return "stub runtime error"; }

hipError_t hipEventCreate(hipEvent_t* event) {
  static int token;
  *event = reinterpret_cast<hipEvent_t>(&token);
  return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }

hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }

hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}

// Graphs: handles that stand for nothing; a launch runs no kernel.
static int graph_token;
// The tile-ordering kernel has a token of its own, so that the nodes that
// launch it can be counted: how many since the last query, and the grid
// and list length (its third argument) of the last one.
static int order_token;
static int order_nodes = 0, order_last_n = -1, order_last_grid = 0;

int stub_order_nodes(int* last_n, int* last_grid) {
  const int k = order_nodes;
  *last_n = order_last_n;
  *last_grid = order_last_grid;
  order_nodes = 0;
  order_last_n = -1;
  order_last_grid = 0;
  return k;
}

hipError_t hipGraphCreate(hipGraph_t* pGraph, unsigned int) {
  *pGraph = reinterpret_cast<hipGraph_t>(&graph_token);
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

hipError_t hipGraphAddKernelNode(hipGraphNode_t* pGraphNode, hipGraph_t,
                                 const hipGraphNode_t*, size_t,
                                 const hipKernelNodeParams* p) {
  if (p && p->func == &order_token) {
    ++order_nodes;
    order_last_n = *static_cast<const int*>(p->kernelParams[2]);
    order_last_grid = (int)p->gridDim.x;
  }
  *pGraphNode = reinterpret_cast<hipGraphNode_t>(&graph_token);
  return hipSuccess;
}

hipError_t hipGraphAddEventRecordNode(hipGraphNode_t* pGraphNode, hipGraph_t,
                                      const hipGraphNode_t*, size_t,
                                      hipEvent_t) {
  *pGraphNode = reinterpret_cast<hipGraphNode_t>(&graph_token);
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* pGraphExec, hipGraph_t,
                               hipGraphNode_t*, char*, size_t) {
  *pGraphExec = reinterpret_cast<hipGraphExec_t>(&graph_token);
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }

hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }

}  // extern "C"

namespace tr {

static int kernel_token;

hipError_t launch_front(const DevScen*, int, const int4*, int, int, int, int,
                        hipStream_t) {
  return hipSuccess;
}
hipError_t launch_back(const DevScen*, int, const int4*, int, int, int,
                       hipStream_t) {
  return hipSuccess;
}
hipError_t launch_step(const DevScen*, int, const int4*, int, int, bool,
                       hipStream_t) {
  return hipSuccess;
}
void* step_kernel(bool, bool) { return &kernel_token; }
void* front_kernel(bool) { return &kernel_token; }
void* back_kernel(bool) { return &kernel_token; }
void* advance_kernel() { return &kernel_token; }
void* order_kernel() { return &order_token; }
hipError_t launch_advance(DevScen*, const int*, int, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_ring(DevScen*, const int*, int, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_stats(const DevScen*, unsigned long long*, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_export(const DevScen*, ExportBufs, int, int, int, int,
                         hipStream_t) {
  return hipSuccess;
}
// the allocation-free step's fixed scratch, as a host array
static int4 stub_scratch[kScratchWork + kScratchSlots / 4];
hipError_t scratch_init(int) { return hipSuccess; }
void* scratch_ptr(int) { return stub_scratch; }

}  // namespace tr
