// Scratch memory of the allocation-free entry point fm_fine_propagate_noalloc:
// one fixed array in device memory.  Every GPU the library runs on holds its
// own copy (at its own address) for the life of the process.  Host code never
// uses the array's name as an address: the name is a host-side stand-in, so
// the address of each device's copy is looked up once, with that device
// current, and kept.
#include "engine.h"

#include <mutex>

namespace fm {

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};
}  // namespace

// Look up the current device's copy (once per device).  Called at flow
// creation, with the flow's device current.
fm_status noalloc_setup() {
  int dev = -1;
  FM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the allocation-free scratch table holds", dev, kMaxDevices);
    return FM_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[dev]) return FM_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
  if (!p) {
    set_error("hipGetSymbolAddress(scratch) returned a null address");
    return FM_ERR_DEVICE;
  }
  g_ptr[dev] = (char*)p;
  return FM_OK;
}

char* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace fm
