// Caching device allocator behind DArr (the contract is stated where
// PoolBlock is declared).  hipMalloc and hipFree cost tens of microseconds
// each and hipFree waits for the device, while a hierarchy build, an assembly
// and a solver setup each allocate and free a few hundred arrays whose sizes
// repeat from one call to the next.
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"

namespace camfe {
namespace {

typedef std::pair<int, hipStream_t> StreamKey;

std::mutex g_mu;
std::map<StreamKey, int> g_live;                                       // attached streams (reference counts)
std::map<StreamKey, std::map<size_t, std::vector<void*>>> g_cache;     // free blocks per stream and size class
std::map<int, size_t> g_cached_bytes, g_limit;                         // per device
thread_local hipStream_t t_stream = nullptr;

// classes: multiples of 256 B up to 1 MiB, then eight per power of two
size_t size_class(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 255) & ~size_t(255);
  int lg = 63 - __builtin_clzll((unsigned long long)b);
  const size_t q = size_t(1) << (lg - 3);
  return (b + q - 1) / q * q;
}

size_t limit_of(int dev) {   // g_mu held
  auto it = g_limit.find(dev);
  if (it != g_limit.end()) return it->second;
  size_t total_b = 0;
  if (hipDeviceTotalMem(&total_b, dev) != hipSuccess) total_b = 0;
  return g_limit[dev] = total_b / 4;
}

void free_on(int dev, void* p) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != dev) (void)hipSetDevice(dev);
  (void)hipFree(p);
  if (cur != dev) (void)hipSetDevice(cur);
}

// frees every cached block (after an allocation failed)
void trim_all() {
  std::vector<std::pair<int, void*>> victims;
  {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : g_cache)
      for (auto& cl : kv.second)
        for (void* p : cl.second) victims.push_back({kv.first.first, p});
    g_cache.clear();
    g_cached_bytes.clear();
  }
  for (auto& v : victims) free_on(v.first, v.second);
}

}  // namespace

void set_current_stream(hipStream_t st) { t_stream = st; }

void* pool_alloc(size_t bytes, PoolBlock* b) {
  int dev = 0;
  CAMFE_HIP(hipGetDevice(&dev));
  const size_t cls = size_class(bytes);
  const StreamKey key(dev, t_stream);
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_live.count(key)) {
      auto it = g_cache.find(key);
      if (it != g_cache.end()) {
        auto cl = it->second.find(cls);
        if (cl != it->second.end() && !cl->second.empty()) {
          void* p = cl->second.back();
          cl->second.pop_back();
          g_cached_bytes[dev] -= cls;
          *b = PoolBlock{cls, dev, t_stream};
          return p;
        }
      }
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_all();
    CAMFE_HIP(hipMalloc(&p, cls));
  }
  *b = PoolBlock{cls, dev, t_stream};
  return p;
}

void pool_free(void* p, const PoolBlock& b) {
  {
    std::lock_guard<std::mutex> g(g_mu);
    const StreamKey key(b.dev, b.st);
    if (g_live.count(key) && g_cached_bytes[b.dev] + b.cls <= limit_of(b.dev)) {
      g_cache[key][b.cls].push_back(p);
      g_cached_bytes[b.dev] += b.cls;
      return;
    }
  }
  free_on(b.dev, p);
}

void pool_attach_stream(int dev, hipStream_t st) {
  std::lock_guard<std::mutex> g(g_mu);
  g_live[StreamKey(dev, st)]++;
}

void pool_detach_stream(int dev, hipStream_t st) {
  std::vector<void*> victims;
  {
    std::lock_guard<std::mutex> g(g_mu);
    const StreamKey key(dev, st);
    auto it = g_live.find(key);
    if (it == g_live.end() || --it->second > 0) return;
    g_live.erase(it);
    auto c = g_cache.find(key);
    if (c != g_cache.end()) {
      for (auto& cl : c->second)
        for (void* p : cl.second) {
          victims.push_back(p);
          g_cached_bytes[dev] -= cl.first;
        }
      g_cache.erase(c);
    }
  }
  for (void* p : victims) free_on(dev, p);
}

}  // namespace camfe
