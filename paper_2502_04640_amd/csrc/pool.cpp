// Device memory pool of libxm (declared in common.h).
//
// A build of the 10155-frame workload holds ~20 GB of device memory (Q in two
// precisions, the grounded-Laplacian inverse, the elimination products, sort
// buffers).  Taking that from the runtime on every build and giving it back on
// every free costs tens to thousands of milliseconds per call, so freed blocks
// are kept per device, keyed by size, and handed out again to requests of about
// the same size.  A block is recycled only after the device has gone idle (the
// ordering hipFree gives), so no kernel still in flight can see it reused.
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace xm {
namespace {

struct Block {
  size_t bytes;
  int dev;
};

struct Pool {
  std::mutex mu;
  std::unordered_map<void*, Block> live;
  std::map<int, std::multimap<size_t, void*>> cache;  // device -> (block bytes -> block)
  size_t live_bytes = 0, cached_bytes = 0;
};

// Never destroyed: buffers owned by static objects of a caller may be freed
// after this translation unit's statics would have been torn down.
Pool& pool() {
  static Pool* p = new Pool();
  return *p;
}

// Size classes: 256 B up to 1 MiB, 2 MiB above (the runtime's large-page size).
size_t size_class(size_t b) {
  if (b <= (size_t(1) << 20)) return round_up(b, 256);
  return round_up(b, size_t(2) << 20);
}

// Most bytes kept in cached blocks (over all devices); XM_POOL_CACHE_GB
// overrides the default of 64 GiB.
size_t cache_limit() {
  static const size_t lim = [] {
    const char* e = std::getenv("XM_POOL_CACHE_GB");
    const double gb = e ? std::atof(e) : 64.0;
    return static_cast<size_t>((gb > 0 ? gb : 0.0) * double(size_t(1) << 30));
  }();
  return lim;
}

struct DeviceScope {  // make `dev` current for the scope
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Release cached blocks of `dev` (all of them when dev < 0) until at most
// `keep` cached bytes remain overall, largest first.  Caller holds the lock.
size_t evict_locked(Pool& P, int dev, size_t keep) {
  size_t freed = 0;
  for (auto& kv : P.cache) {
    if (dev >= 0 && kv.first != dev) continue;
    auto& m = kv.second;
    DeviceScope scope(kv.first);
    while (!m.empty() && P.cached_bytes > keep) {
      auto it = std::prev(m.end());
      (void)hipFree(it->second);
      P.cached_bytes -= it->first;
      freed += it->first;
      m.erase(it);
    }
  }
  return freed;
}

}  // namespace

void* pool_alloc(size_t bytes) {
  Pool& P = pool();
  const size_t b = size_class(bytes);
  int dev = 0;
  XM_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto& m = P.cache[dev];
    auto it = m.lower_bound(b);
    // reuse a cached block of at most 1.25x the request
    if (it != m.end() && it->first <= b + b / 4) {
      void* ptr = it->second;
      const size_t got = it->first;
      m.erase(it);
      P.cached_bytes -= got;
      P.live[ptr] = Block{got, dev};
      P.live_bytes += got;
      return ptr;
    }
  }
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, b);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> g(P.mu);
      evict_locked(P, dev, 0);
    }
    e = hipMalloc(&ptr, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(XM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                 hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> g(P.mu);
  P.live[ptr] = Block{b, dev};
  P.live_bytes += b;
  return ptr;
}

void pool_free(void* ptr) {
  if (!ptr) return;
  Pool& P = pool();
  Block blk{0, 0};
  {
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(ptr);
    if (it == P.live.end()) return;  // not ours: nothing to do
    blk = it->second;
    P.live.erase(it);
    P.live_bytes -= blk.bytes;
  }
  {
    // work still queued on the device may use the block
    DeviceScope scope(blk.dev);
    (void)hipDeviceSynchronize();
  }
  std::lock_guard<std::mutex> g(P.mu);
  P.cache[blk.dev].emplace(blk.bytes, ptr);
  P.cached_bytes += blk.bytes;
  if (P.cached_bytes > cache_limit()) evict_locked(P, -1, cache_limit());
}

size_t pool_trim() {
  Pool& P = pool();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(P.mu);
  return evict_locked(P, -1, 0);
}

void pool_usage(size_t* live, size_t* cached) {
  Pool& P = pool();
  std::lock_guard<std::mutex> g(P.mu);
  if (live) *live = P.live_bytes;
  if (cached) *cached = P.cached_bytes;
}

}  // namespace xm
