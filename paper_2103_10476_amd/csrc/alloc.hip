// Device memory for the library: a stream-ordered caching allocator, and pinned host staging
// for small readbacks.
//
// Setup allocates and frees a few hundred buffers per level; done with hipMallocAsync /
// hipFreeAsync each call costs tens of microseconds of host time and leaves the GPU idle.
// Blocks are instead taken from hipMalloc once, rounded to a size class, and kept in a free
// list per (device, stream) when released.  A block freed on stream s is only handed out
// again for work on the same stream s, so stream order alone guarantees that every kernel
// that used it has finished before its next owner's kernels start; no event is needed.
// When hipMalloc fails, every cached block is returned to the driver (after a device
// synchronisation) and the allocation is retried once.
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.hpp"

namespace sa {

namespace {

struct Cache {
  std::mutex mu;
  // (device, stream) -> size -> free blocks of that size
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> free_lists;
  struct Live {
    size_t size;
    int dev;
    Meter *meter;
  };
  std::unordered_map<void *, Live> live;
  size_t cached = 0, in_use = 0;
};

Cache &cache() {
  static Cache *c = new Cache;  // never destroyed: blocks may be released at process exit
  return *c;
}

// Size classes: multiples of 256 B up to 4 KiB, then 8 classes per power of two (at most
// 12.5% over the request).
size_t size_class(size_t b) {
  if (b <= 4096) return (b + 255) & ~size_t(255);
  size_t p = size_t(1) << (63 - __builtin_clzll(b));
  const size_t step = p / 8;
  return (b + step - 1) / step * step;
}

void release_cached_locked(Cache &c) {
  for (auto &kv : c.free_lists)
    for (auto &blk : kv.second) (void)hipFree(blk.second);
  c.free_lists.clear();
  c.cached = 0;
}

thread_local Meter *t_meter = nullptr;

void meter_add(Meter *m, int64_t sz) {
  for (; m; m = m->parent) {
    m->live += sz;
    if (m->live > m->peak) m->peak = m->live;
  }
}

}  // namespace

void meter_begin(Meter *m) { t_meter = m; }
void meter_end() { t_meter = nullptr; }

void *dev_alloc(size_t bytes, hipStream_t s) {
  Cache &c = cache();
  int dev = 0;
  SA_HIP(hipGetDevice(&dev));
  const size_t sz = size_class(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto fl = c.free_lists.find({dev, s});
    if (fl != c.free_lists.end()) {
      // the same class, or the next one up (at most ~25% larger)
      auto it = fl->second.lower_bound(sz);
      if (it != fl->second.end() && it->first <= sz + sz / 4) {
        void *p = it->second;
        const size_t got = it->first;
        fl->second.erase(it);
        c.cached -= got;
        c.in_use += got;
        c.live[p] = {got, dev, t_meter};
        meter_add(t_meter, (int64_t)got);
        return p;
      }
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(c.mu);
    (void)hipDeviceSynchronize();
    release_cached_locked(c);
    e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(SA_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  std::lock_guard<std::mutex> lk(c.mu);
  c.in_use += sz;
  c.live[p] = {sz, dev, t_meter};
  meter_add(t_meter, (int64_t)sz);
  return p;
}

void dev_free(void *p, hipStream_t s) {
  if (!p) return;
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;  // not ours: ignore
  const size_t sz = it->second.size;
  const int dev = it->second.dev;
  meter_add(it->second.meter, -(int64_t)sz);
  c.live.erase(it);
  c.in_use -= sz;
  c.cached += sz;
  c.free_lists[{dev, s}].emplace(sz, p);
}

void meter_read(const Meter *m, int64_t *live, int64_t *peak) {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (live) *live = m->live;
  if (peak) *peak = m->peak;
}

void dev_release_stream(hipStream_t s) {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  auto fl = c.free_lists.find({dev, s});
  if (fl == c.free_lists.end()) return;
  (void)hipStreamSynchronize(s);
  for (auto &blk : fl->second) {
    (void)hipFree(blk.second);
    c.cached -= blk.first;
  }
  c.free_lists.erase(fl);
}

void dev_release_cached() {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  (void)hipDeviceSynchronize();
  release_cached_locked(c);
}

void dev_cache_stats(size_t *in_use, size_t *cached) {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (in_use) *in_use = c.in_use;
  if (cached) *cached = c.cached;
}

// ---- pinned staging for readbacks ---------------------------------------------------------
// Copies into pageable host memory go through a driver bounce buffer and cost ~100 us each;
// each thread stages readbacks in a pinned buffer of its own instead.  Buffers are recycled
// through a process-wide list when their thread ends (no HIP call at thread exit).  A second
// per-thread buffer, coherent (fine-grained: kernels' system-scope stores reach it without a
// synchronise), holds status words that the thread polls while kernels run.
namespace {
struct PinnedPool {
  std::mutex mu;
  std::vector<std::pair<void *, size_t>> spare[2];  // [0] default, [1] coherent
};
PinnedPool &pinned_pool() {
  static PinnedPool *p = new PinnedPool;
  return *p;
}
struct PinnedHolder {
  int kind;  // 0 default, 1 coherent
  void *p = nullptr;
  size_t n = 0;
  explicit PinnedHolder(int k) : kind(k) {}
  ~PinnedHolder() {
    if (!p) return;
    PinnedPool &pp = pinned_pool();
    std::lock_guard<std::mutex> lk(pp.mu);
    pp.spare[kind].emplace_back(p, n);
  }
};
thread_local PinnedHolder t_pinned(0), t_status(1);

void *pinned_buffer(PinnedHolder &h, size_t bytes) {
  if (h.p && h.n >= bytes) return h.p;
  {
    PinnedPool &pp = pinned_pool();
    std::lock_guard<std::mutex> lk(pp.mu);
    auto &spare = pp.spare[h.kind];
    if (h.p) spare.emplace_back(h.p, h.n);
    h.p = nullptr;
    h.n = 0;
    for (size_t i = 0; i < spare.size(); ++i)
      if (spare[i].second >= bytes) {
        h.p = spare[i].first;
        h.n = spare[i].second;
        spare.erase(spare.begin() + (ptrdiff_t)i);
        return h.p;
      }
  }
  size_t n = 4096;
  while (n < bytes) n *= 2;
  void *p = nullptr;
  SA_HIP(hipHostMalloc(&p, n, h.kind ? hipHostMallocCoherent : hipHostMallocDefault));
  h.p = p;
  h.n = n;
  return p;
}
}  // namespace

void *pinned_staging(size_t bytes) { return pinned_buffer(t_pinned, bytes); }
void *pinned_status(size_t bytes) { return pinned_buffer(t_status, bytes); }

// Small readbacks: one workgroup copies the words straight into the pinned staging buffer
// through its device mapping (cheaper than the runtime's copy kernel for a few bytes).
__global__ void k_copy_words(uint32_t *dst, const uint32_t *src, int32_t nw) {
  for (int32_t i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
}

void readback(void *host, const void *dev, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes > (size_t(1) << 20)) {  // bulk copies: straight into the caller's memory
    SA_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    return;
  }
  void *st = pinned_staging(bytes);
  if (bytes <= 4096 && bytes % 4 == 0 && (uintptr_t)dev % 4 == 0) {
    void *dst = nullptr;
    SA_HIP(hipHostGetDevicePointer(&dst, st, 0));
    k_copy_words<<<1, kBlock, 0, s>>>((uint32_t *)dst, (const uint32_t *)dev,
                                      (int32_t)(bytes / 4));
    SA_LAUNCH_CHECK();
  } else {
    SA_HIP(hipMemcpyAsync(st, dev, bytes, hipMemcpyDeviceToHost, s));
  }
  SA_HIP(hipStreamSynchronize(s));
  std::memcpy(host, st, bytes);
}

}  // namespace sa
