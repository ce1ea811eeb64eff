// scratch.hip -- the fixed device scratch of the allocation-free step entry
// point: the work list of one call (tiles of every listed slot, dealt to the
// XCDs) and its slot list, in a file-scope device array instead of memory
// the context allocates.  Each GPU the library runs on holds its own copy
// until the process ends; its address on a device is looked up once, with
// that device current, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace tr {

namespace {

// work items, then the slot list packed four per int4
constexpr int kScratchInt4 = kScratchWork + kScratchSlots / 4;
static __device__ __align__(256) int4 scratch[kScratchInt4];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // caller makes it current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace tr
