// Device memory pool of the library.
//
// The builder needs a few dozen temporary arrays (up to several times nnz
// bytes), and every handle owns its format arrays.  hipMalloc of large blocks
// maps pages and hipFree synchronises the device, so building a format with
// plain hipMalloc/hipFree spends milliseconds outside the kernels.  This pool
// keeps freed blocks per device and hands them out again.
//
// Ordering: a block freed with a stream records an event on that stream; the
// next allocation that reuses the block makes its own stream wait for that
// event, so work queued on the old stream finishes before the new owner's work
// starts.  A block freed without a stream must be idle already.
//
// A failed hipMalloc first returns every cached block of the device to HIP and
// tries again.  TC_POOL=0 in the environment turns caching off.
//
// Host blocks (the build's page-locked transfer buffers, a handle's workload
// list) are kept the same way, so repeated builds neither page-lock nor fault
// in fresh host memory.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <new>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "tc_internal.h"

namespace tc {
namespace {

struct Cached {
  void* p;
  size_t bytes;
  hipEvent_t ev;  // null: idle
};

struct Live {
  size_t bytes;
  int dev;
};

struct Pool {
  std::mutex mu;
  std::unordered_map<int, std::multimap<size_t, Cached>> free_by_dev;
  std::unordered_map<void*, Live> live;
  size_t cached_bytes = 0;
  int enabled = -1;
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: HIP may be gone at exit
  return *p;
}

size_t round_size(size_t b) {
  if (b <= ((size_t)1 << 20)) return (b + 511) & ~(size_t)511;
  const size_t g = (size_t)2 << 20;
  return (b + g - 1) / g * g;
}

void release_block(Cached& c) {
  if (c.ev) {
    (void)hipEventSynchronize(c.ev);
    (void)hipEventDestroy(c.ev);
  }
  (void)hipFree(c.p);
}

void trim_device(Pool& P, int dev) {
  auto it = P.free_by_dev.find(dev);
  if (it == P.free_by_dev.end()) return;
  for (auto& kv : it->second) {
    P.cached_bytes -= kv.second.bytes;
    release_block(kv.second);
  }
  it->second.clear();
}

}  // namespace

void* pool_alloc(size_t bytes, hipStream_t st) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (P.enabled < 0) {
    const char* e = std::getenv("TC_POOL");
    P.enabled = (e && e[0] == '0') ? 0 : 1;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const size_t need = round_size(bytes == 0 ? 1 : bytes);
  if (P.enabled) {
    auto& fl = P.free_by_dev[dev];
    auto it = fl.lower_bound(need);
    // best fit, but do not hand a large block to a much smaller request
    if (it != fl.end() && it->first <= need + need / 4 + ((size_t)2 << 20)) {
      Cached c = it->second;
      fl.erase(it);
      P.cached_bytes -= c.bytes;
      if (c.ev) {
        if (hipStreamWaitEvent(st, c.ev, 0) != hipSuccess) (void)hipEventSynchronize(c.ev);
        (void)hipEventDestroy(c.ev);
      }
      P.live[c.p] = Live{c.bytes, dev};
      return c.p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    trim_device(P, dev);
    p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  P.live[p] = Live{need, dev};
  return p;
}

void pool_free(void* p, hipStream_t st, bool idle) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live.find(p);
  if (it == P.live.end()) {
    (void)hipFree(p);
    return;
  }
  const Live l = it->second;
  P.live.erase(it);
  if (!P.enabled) {
    (void)hipFree(p);
    return;
  }
  Cached c{p, l.bytes, nullptr};
  if (!idle) {
    if (hipEventCreateWithFlags(&c.ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(c.ev, st) != hipSuccess) {
      (void)hipGetLastError();
      if (c.ev) (void)hipEventDestroy(c.ev);
      (void)hipFree(p);
      return;
    }
  }
  P.free_by_dev[l.dev].emplace(l.bytes, c);
  P.cached_bytes += l.bytes;
}

size_t pool_release_cached() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  size_t freed = P.cached_bytes;
  for (auto& kv : P.free_by_dev) {
    for (auto& b : kv.second) release_block(b.second);
    kv.second.clear();
  }
  P.cached_bytes = 0;
  return freed;
}

size_t pool_cached_bytes() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  return P.cached_bytes;
}

namespace {
bool pool_enabled() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (P.enabled < 0) {
    const char* e = std::getenv("TC_POOL");
    P.enabled = (e && e[0] == '0') ? 0 : 1;
  }
  return P.enabled != 0;
}

struct HostPoolState {
  std::mutex mu;
  std::vector<HostBlock> free_blocks;
};
HostPoolState& host_pool() {
  static HostPoolState* p = new HostPoolState();  // never destroyed, like the device pool
  return *p;
}
void host_free_block(const HostBlock& b) {
  if (b.pinned)
    (void)hipHostFree(b.p);
  else
    std::free(b.p);
}
}  // namespace

HostBlock host_take(size_t bytes, bool pinned) {
  HostPoolState& P = host_pool();
  if (pool_enabled()) {
    std::lock_guard<std::mutex> lk(P.mu);
    size_t best = P.free_blocks.size();
    for (size_t i = 0; i < P.free_blocks.size(); ++i) {
      const HostBlock& c = P.free_blocks[i];
      // best fit, but not a block much larger than the request
      if (c.pinned == pinned && c.cap >= bytes && c.cap <= bytes + bytes / 4 + ((size_t)2 << 20) &&
          (best == P.free_blocks.size() || c.cap < P.free_blocks[best].cap))
        best = i;
    }
    if (best < P.free_blocks.size()) {
      const HostBlock b = P.free_blocks[best];
      P.free_blocks.erase(P.free_blocks.begin() + (std::ptrdiff_t)best);
      return b;
    }
  }
  HostBlock b;
  b.cap = round_size(bytes);
  if (pinned && hipHostMalloc(&b.p, b.cap, hipHostMallocDefault) == hipSuccess) {
    b.pinned = true;
    return b;
  }
  if (pinned) (void)hipGetLastError();  // pageable memory stands in
  b.p = std::malloc(b.cap);
  if (!b.p) throw std::bad_alloc();
  return b;
}

void host_give(const HostBlock& b) {
  if (!b.p) return;
  if (!pool_enabled()) {
    host_free_block(b);
    return;
  }
  HostPoolState& P = host_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  P.free_blocks.push_back(b);
}

size_t host_release_cached() {
  HostPoolState& P = host_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  size_t freed = 0;
  for (const HostBlock& b : P.free_blocks) {
    freed += b.cap;
    host_free_block(b);
  }
  P.free_blocks.clear();
  return freed;
}

}  // namespace tc
