// Device memory cache (see pool.h).
#include "pool.h"

#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.h"

namespace hps {

namespace {

constexpr size_t kSmall = size_t(1) << 20;      // below: 512-byte granularity
constexpr size_t kLargeGrain = size_t(2) << 20;  // above: 2 MiB granularity
constexpr size_t kMaxCached = size_t(64) << 30;  // beyond this, released blocks are freed

struct Pool {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void*> free_;          // (device, size) -> block
  std::unordered_map<void*, std::pair<int, size_t>> live_;    // block -> (device, size)
  size_t cached = 0, in_use = 0;
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: no HIP calls during static teardown
  return *p;
}

size_t round_size(size_t b) {
  if (b == 0) b = 1;
  if (b < kSmall) return (b + 511) & ~size_t(511);
  return (b + kLargeGrain - 1) / kLargeGrain * kLargeGrain;
}

size_t trim_locked(Pool& P) {
  size_t freed = 0;
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : P.free_) {
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
    freed += kv.first.second;
  }
  (void)hipSetDevice(cur);
  P.free_.clear();
  P.cached = 0;
  return freed;
}

}  // namespace

void* pool_alloc(size_t bytes) {
  Pool& P = pool();
  const size_t r = round_size(bytes);
  int dev = 0;
  HPS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(P.mu);
  // Best fit among cached blocks of this device, wasting at most a quarter.
  auto it = P.free_.lower_bound({dev, r});
  if (it != P.free_.end() && it->first.first == dev && it->first.second <= r + r / 4) {
    void* p = it->second;
    const size_t sz = it->first.second;
    P.free_.erase(it);
    P.cached -= sz;
    P.live_[p] = {dev, sz};
    P.in_use += sz;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e == hipErrorOutOfMemory && !P.free_.empty()) {
    (void)hipGetLastError();
    trim_locked(P);
    e = hipMalloc(&p, r);
  }
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? HPS_ENOMEM : HPS_EDEVICE,
                std::string("hipMalloc of ") + std::to_string(r) + " bytes: " + hipGetErrorString(e));
  P.live_[p] = {dev, r};
  P.in_use += r;
  return p;
}

void pool_release(void* p) {
  if (!p) return;
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.live_.find(p);
  if (it == P.live_.end()) return;  // not ours: nothing to do
  const auto [dev, sz] = it->second;
  P.live_.erase(it);
  P.in_use -= sz;
  if (P.cached + sz > kMaxCached) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(dev);
    (void)hipFree(p);
    (void)hipSetDevice(cur);
    return;
  }
  P.free_.insert({{dev, sz}, p});
  P.cached += sz;
}

size_t pool_trim() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  return trim_locked(P);
}

void pool_stats(size_t* cached, size_t* in_use) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  if (cached) *cached = P.cached;
  if (in_use) *in_use = P.in_use;
}

}  // namespace hps
