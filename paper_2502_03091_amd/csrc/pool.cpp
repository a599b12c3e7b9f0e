// Process-wide cache of device allocations behind DevBuf.
//
// A multigrid setup is repeated many times on one lattice shape (once per gauge
// configuration), and its large buffers (test vectors, residuals, prolongator,
// coarse links: hundreds of GB at 48^3x96) are expensive to obtain and give
// back once device memory has been recycled: after earlier frees, a single
// hipMalloc of tens of GB has taken seconds on MI355X, and so has the hipFree
// of such a buffer.  Freed buffers are therefore kept per device and handed to
// a later request of about the same size (at most 1/8 larger, or 2 MiB for
// small requests).  When hipMalloc does not fit, the device's cache is given
// back and the allocation retried; crk_release_cached_memory gives it back on
// request.
//
// Contents of a reused buffer are whatever its last owner left: every user
// writes (or clears) what it reads.  A free waits for the device, as hipFree
// does, so that no queued kernel can still touch a buffer another request is
// given.
#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace crk {

namespace {

struct Block {
  int dev;
  size_t bytes;
};

struct Pool {
  std::mutex mu;
  std::unordered_map<void*, Block> live;
  std::map<int, std::multimap<size_t, void*>> cached;
  std::map<int, size_t> cached_bytes;
};

// Never destroyed: buffers owned by static objects may be freed during exit.
Pool& pool() {
  static Pool* p = new Pool;
  return *p;
}

size_t round_request(size_t n) {
  const size_t g = n < (size_t(1) << 20) ? size_t(4096) : size_t(2) << 20;
  return (n + g - 1) / g * g;
}

size_t slack(size_t n) { return std::max(n / 8, size_t(2) << 20); }

// Runs f with device `dev` current and restores the caller's device.
template <class F> void on_device(int dev, F&& f) {
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != dev) (void)hipSetDevice(dev);
  f();
  if (cur != dev && cur >= 0) (void)hipSetDevice(cur);
}

void release_device(int dev) {
  std::vector<void*> blocks;
  {
    std::lock_guard<std::mutex> g(pool().mu);
    auto& c = pool().cached[dev];
    for (auto& kv : c) blocks.push_back(kv.second);
    c.clear();
    pool().cached_bytes[dev] = 0;
  }
  if (blocks.empty()) return;
  on_device(dev, [&] {
    for (void* p : blocks) (void)hipFree(p);
    (void)hipGetLastError();
  });
}

}  // namespace

void* device_alloc(size_t n) {
  if (n == 0) return nullptr;
  const size_t r = round_request(n);
  int dev = 0;
  CRK_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(pool().mu);
    auto& c = pool().cached[dev];
    auto it = c.lower_bound(r);
    if (it != c.end() && it->first <= r + slack(r)) {
      void* p = it->second;
      const size_t sz = it->first;
      c.erase(it);
      pool().cached_bytes[dev] -= sz;
      pool().live[p] = Block{dev, sz};
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    release_device(dev);
    e = hipMalloc(&p, r);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? CRK_ENOMEM : CRK_EHIP,
         "hipMalloc(" + std::to_string(r) + " bytes): " + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> g(pool().mu);
  pool().live[p] = Block{dev, r};
  return p;
}

void device_free(void* p) noexcept {
  if (!p) return;
  Block b{};
  {
    std::lock_guard<std::mutex> g(pool().mu);
    auto it = pool().live.find(p);
    if (it == pool().live.end()) return;
    b = it->second;
    pool().live.erase(it);
  }
  hipError_t e = hipSuccess;
  on_device(b.dev, [&] { e = hipDeviceSynchronize(); });
  if (e != hipSuccess) {  // the device is in error: do not hand the buffer out again
    (void)hipGetLastError();
    on_device(b.dev, [&] { (void)hipFree(p); (void)hipGetLastError(); });
    return;
  }
  std::lock_guard<std::mutex> g(pool().mu);
  pool().cached[b.dev].insert({b.bytes, p});
  pool().cached_bytes[b.dev] += b.bytes;
}

size_t device_cached_bytes(int dev) {
  std::lock_guard<std::mutex> g(pool().mu);
  auto it = pool().cached_bytes.find(dev);
  return it == pool().cached_bytes.end() ? 0 : it->second;
}

size_t device_free_bytes() {
  int dev = 0;
  CRK_HIP(hipGetDevice(&dev));
  size_t fr = 0, tot = 0;
  CRK_HIP(hipMemGetInfo(&fr, &tot));
  return fr + device_cached_bytes(dev);
}

void device_release_cached() {
  std::vector<int> devs;
  {
    std::lock_guard<std::mutex> g(pool().mu);
    for (auto& kv : pool().cached) devs.push_back(kv.first);
  }
  for (int d : devs) release_device(d);
}

}  // namespace crk
