// Device-memory pools of the contexts: cached blocks keyed by size class, a
// reserve left free for the runtime, and the return of other contexts'
// cached blocks when the device runs short.  Plain C++ on top of the raw
// allocation calls of kernels.h (HIP in kernels.hip).
#include <algorithm>
#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace sadmrg {

[[noreturn]] void dev_fail_nomem(const char* what);  // defined by the engine (throws)

// ---------------------------------------------------------------------------
// Device memory.  Without a bound pool, dev_alloc/dev_free are the raw device
// allocation calls.  A context binds its own pool for the duration of every call: freed
// blocks are kept (keyed by a size class) and handed out again, so the
// per-micro-iteration stores and plans do not pay a device allocation and
// release (which synchronises the device) every step.  A context uses one stream at a time,
// so a block reused on it is ordered after every earlier use.
// ---------------------------------------------------------------------------
struct DevPool {
  std::multimap<size_t, void*> cached;     // size class -> block
  std::unordered_map<void*, size_t> owned;  // every block of this pool -> size class
  size_t cached_bytes = 0;
  std::mutex mu;  // host threads of one context may share the pool
  // caller-supplied allocator (null: dev_raw_alloc / dev_raw_free)
  DevAllocFn alloc_fn = nullptr;
  DevFreeFn free_fn = nullptr;
  void* user = nullptr;
  int device = 0;
};
// a new block for `pool` (its allocator, else the raw call); null on failure
static void* pool_raw_alloc(DevPool* pool, size_t bytes) {
  if (pool && pool->alloc_fn) return pool->alloc_fn(bytes, pool->device, pool->user);
  return dev_raw_alloc(bytes);
}
static void pool_raw_free(DevPool* pool, void* p, size_t bytes) {
  if (pool && pool->free_fn)
    pool->free_fn(p, bytes, pool->device, pool->user);
  else
    dev_raw_free(p);
}
static thread_local DevPool* tl_pool = nullptr;
static constexpr size_t POOL_CACHE_MAX = (size_t)96 << 30;
// Every live pool, so that an allocation that fails in one context can take
// back the blocks the other contexts keep cached.  Lock order: the registry
// before a pool; no thread waits for the registry while holding a pool.
static std::mutex g_pools_mu;
static std::vector<DevPool*> g_pools;

DevPool* dev_pool_create() {
  DevPool* pool = new DevPool();
  std::lock_guard<std::mutex> lk(g_pools_mu);
  g_pools.push_back(pool);
  return pool;
}
void dev_pool_destroy(DevPool* pool) {
  if (!pool) return;
  {
    std::lock_guard<std::mutex> lk(g_pools_mu);
    g_pools.erase(std::remove(g_pools.begin(), g_pools.end(), pool), g_pools.end());
  }
  for (auto& [p, sz] : pool->owned) pool_raw_free(pool, p, sz);
  delete pool;
}
bool dev_pool_set_allocator(DevPool* pool, DevAllocFn a, DevFreeFn f, void* user, int device) {
  if (!pool) return false;
  std::lock_guard<std::mutex> lk(pool->mu);
  if (!pool->owned.empty()) return false;  // blocks of the previous allocator are live
  pool->alloc_fn = a;
  pool->free_fn = f;
  pool->user = user;
  pool->device = device;
  return true;
}
DevPool* dev_pool_bind(DevPool* pool) {
  DevPool* prev = tl_pool;
  tl_pool = pool;
  return prev;
}
DevPool* dev_pool_current() { return tl_pool; }

// size classes: multiples of 256 B up to 64 KiB, then 2^k * {1, 5/4, 3/2, 7/4}
static size_t size_class(size_t b) {
  if (b <= 65536) return (b + 255) & ~(size_t)255;
  size_t p = 65536;
  while (p * 2 < b) p *= 2;
  for (size_t q = 4; q <= 8; ++q)
    if (p / 4 * q >= b) return p / 4 * q;
  return p * 2;
}

static void pool_trim(DevPool* pool, size_t keep) {
  while (pool->cached_bytes > keep && !pool->cached.empty()) {
    auto it = std::prev(pool->cached.end());  // largest first
    pool->cached_bytes -= it->first;
    pool->owned.erase(it->second);
    pool_raw_free(pool, it->second, it->first);
    pool->cached.erase(it);
  }
}
// empty the caches of every pool but `self` (called without holding any
// pool's lock); returns the bytes given back
static size_t trim_other_pools(DevPool* self) {
  size_t freed = 0;
  std::lock_guard<std::mutex> reg(g_pools_mu);
  for (DevPool* q : g_pools) {
    if (q == self) continue;
    std::lock_guard<std::mutex> lk(q->mu);
    freed += q->cached_bytes;
    pool_trim(q, 0);
  }
  return freed;
}

// Device memory the library leaves free for the runtime (kernel scratch,
// queues, code objects, signals): a new block of 1 MiB or more that would cut
// into it first takes back cached blocks, its own pool's and then the other
// contexts', and otherwise fails as out of memory (an error the caller can
// handle, where a runtime allocation failing later would end the queue).
static constexpr size_t DEV_RESERVE = (size_t)6 << 30;
static bool dev_room(size_t bytes) {
  if (bytes < ((size_t)1 << 20)) return true;
  size_t fr = 0, tot = 0;
  if (!dev_raw_meminfo(&fr, &tot)) return true;
  return fr >= bytes + DEV_RESERVE;
}

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  DevPool* pool = tl_pool;
  std::unique_lock<std::mutex> lk;
  if (pool) lk = std::unique_lock<std::mutex>(pool->mu);
  if (pool) {
    bytes = size_class(bytes);
    auto it = pool->cached.find(bytes);
    if (it != pool->cached.end()) {
      void* p = it->second;
      pool->cached.erase(it);
      pool->cached_bytes -= bytes;
      return p;
    }
  }
  if (!dev_room(bytes)) {
    if (pool) pool_trim(pool, 0);
    if (!dev_room(bytes)) {
      if (lk.owns_lock()) lk.unlock();
      trim_other_pools(pool);
      if (pool) lk.lock();
      if (!dev_room(bytes)) dev_fail_nomem("out of device memory (the runtime's reserve is reached)");
    }
  }
  void* p = pool_raw_alloc(pool, bytes);
  if (!p && pool && pool->cached_bytes) {  // give the cache back and retry
    pool_trim(pool, 0);
    p = pool_raw_alloc(pool, bytes);
  }
  if (!p) {  // then the caches of the other contexts
    if (lk.owns_lock()) lk.unlock();
    if (trim_other_pools(pool) > 0) p = pool_raw_alloc(pool, bytes);
    if (pool) lk.lock();
  }
  if (!p) dev_fail_nomem("device allocation failed: out of device memory");
  if (pool) pool->owned[p] = bytes;
  return p;
}
// a block that `pool` owns goes back to its cache (false: not this pool's)
static bool pool_take_back(DevPool* pool, void* p) {
  std::lock_guard<std::mutex> lk(pool->mu);
  auto it = pool->owned.find(p);
  if (it == pool->owned.end()) return false;
  pool->cached.emplace(it->second, p);
  pool->cached_bytes += it->second;
  if (pool->cached_bytes > POOL_CACHE_MAX) pool_trim(pool, POOL_CACHE_MAX / 2);
  return true;
}
void dev_free(void* p) {
  if (!p) return;
  DevPool* pool = tl_pool;
  if (pool && pool_take_back(pool, p)) return;
  {
    // a block of another context's pool, freed on a thread bound to another
    // pool or none (a batch's buffers released while an error unwinds): back
    // to the pool that owns it, which would otherwise free it a second time
    // when it is destroyed
    std::lock_guard<std::mutex> reg(g_pools_mu);
    for (DevPool* q : g_pools)
      if (q != pool && pool_take_back(q, p)) return;
  }
  dev_raw_free(p);
}

}  // namespace sadmrg
