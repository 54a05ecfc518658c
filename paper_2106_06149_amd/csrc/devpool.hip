// Process-wide cache of device allocations.
//
// A context allocates tens of GB (amplitudes, couplings, orbital-pair blocks)
// and frees them when it is destroyed; a caller that builds a new context per
// geometry step would otherwise pay hipMalloc/hipFree of those buffers every
// step, and the driver's cost for mapping and unmapping them varies from
// milliseconds to seconds.  Freed blocks are kept per device and handed out
// again for requests of the same size class.
//
// Size classes: requests up to 1 MiB round up to 512 bytes, larger ones to 2 MiB.
// A cached block serves a request when its size is at least the rounded request
// and at most 1/8 (and 2 MiB) larger.  When hipMalloc fails the device's cache is
// released and the allocation retried once.
//
// Blocks keep whatever the last user wrote; no kernel of the library may rely on
// fresh memory being zero.  With OSV_POOL_POISON set in the environment every
// block handed out is filled with 0xFF bytes (NaN as FP64) to show any such
// reliance; the fill has completed on the device when the block is handed out.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "osv_internal.h"

namespace osv {
namespace {

struct Block {
  size_t size;
  int dev;
};

std::mutex g_mu;
std::unordered_map<void *, Block> g_live;              // handed out
std::map<int, std::multimap<size_t, void *>> g_free;    // per device, by size

size_t size_class(size_t bytes) {
  const size_t small = size_t(512), big = size_t(2) << 20;
  if (bytes <= (size_t(1) << 20)) return (bytes + small - 1) / small * small;
  return (bytes + big - 1) / big * big;
}

bool poison() {
  const char *e = std::getenv("OSV_POOL_POISON");
  return e && e[0] && e[0] != '0';
}

// caller holds g_mu
void release_locked(int dev) {
  auto it = g_free.find(dev);
  if (it == g_free.end()) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != dev) (void)hipSetDevice(dev);
  for (auto &kv : it->second) (void)hipFree(kv.second);
  if (cur != dev) (void)hipSetDevice(cur);
  it->second.clear();
}

}  // namespace

hipError_t pool_alloc(void **p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t sz = size_class(bytes == 0 ? 1 : bytes);
  const size_t slack = std::min(sz / 8, size_t(2) << 20);
  void *q = nullptr;
  size_t got = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto &fl = g_free[dev];
    auto it = fl.lower_bound(sz);
    if (it != fl.end() && it->first <= sz + slack) {
      q = it->second;
      got = it->first;
      fl.erase(it);
      g_live[q] = Block{got, dev};
    }
  }
  if (!q) {
    e = hipMalloc(&q, sz);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      {
        std::lock_guard<std::mutex> lk(g_mu);
        release_locked(dev);
      }
      e = hipMalloc(&q, sz);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    got = sz;
    std::lock_guard<std::mutex> lk(g_mu);
    g_live[q] = Block{got, dev};
  }
  if (poison()) {
    // hipMemset runs on the null stream and may return before the fill is done;
    // the block is next written on the caller's stream, which may be a
    // non-blocking stream not ordered after the null stream, so the fill
    // completes before the block is handed out
    e = hipMemset(q, 0xFF, got);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
  }
  *p = q;
  return hipSuccess;
}

void pool_free(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  g_free[it->second.dev].emplace(it->second.size, p);
  g_live.erase(it);
}

void pool_release(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device >= 0) {
    release_locked(device);
    return;
  }
  for (auto &kv : g_free) release_locked(kv.first);
}

size_t pool_cached_bytes(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t n = 0;
  for (auto &kv : g_free)
    if (device < 0 || kv.first == device)
      for (auto &b : kv.second) n += b.first;
  return n;
}

}  // namespace osv
