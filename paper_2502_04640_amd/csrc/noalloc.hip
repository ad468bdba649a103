// Fixed device scratch of xm_spmm_noalloc: a file-scope device array that
// every product of that entry point takes its temporaries from, so that the
// call allocates nothing.  Each device holds its own copy (at its own address)
// from the time the library's code is loaded on it until the process ends.
#include <mutex>

#include "problem.h"

static __device__ __align__(256) char scratch[xm::kNoallocScratchBytes];

namespace xm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_addr[kMaxDevices] = {};

}  // namespace

// Address of the current device's copy of `scratch`.  In host code the array's
// name stands for no device address, so it is looked up once per device with
// hipGetSymbolAddress (that device current) and kept; every later call on the
// device reuses it.
char* noalloc_scratch_base() {
  int dev = -1;
  XM_HIP(hipGetDevice(&dev));
  require(dev >= 0 && dev < kMaxDevices, XM_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[dev] == nullptr) {
    void* ptr = nullptr;
    XM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, XM_EHIP, "hipGetSymbolAddress returned NULL for the fixed scratch");
    g_addr[dev] = static_cast<char*>(ptr);
  }
  return g_addr[dev];
}

}  // namespace xm
