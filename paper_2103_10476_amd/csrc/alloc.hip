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
#include <atomic>
#include <chrono>
#include <cstdlib>
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
// through a process-wide list when their thread ends (no HIP call at thread exit).  Two more
// per-thread buffers are coherent (fine-grained: kernels' system-scope stores reach them
// without a synchronise): one holds status words that the thread polls while kernels run, the
// other the small readbacks, whose arrival the thread sees from a tag word written after them.
namespace {
struct PinnedPool {
  std::mutex mu;
  std::vector<std::pair<void *, size_t>> spare[3];  // [0] default, [1], [2] coherent
};
PinnedPool &pinned_pool() {
  static PinnedPool *p = new PinnedPool;
  return *p;
}
struct PinnedHolder {
  int kind;  // 0 default, 1 and 2 coherent
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
thread_local PinnedHolder t_pinned(0), t_status(1), t_words(2);

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

// Small readbacks: one workgroup copies the words straight into the thread's coherent buffer
// through its device mapping (cheaper than the runtime's copy kernel for a few bytes), then,
// after a system-scope fence, writes the readback's tag; the host polls the tag instead of
// synchronising the stream (~3 us less per readback, and the stream's earlier work is done by
// then: the copy runs after it).
constexpr int32_t kWordsMax = 1024;  // words per small readback; the tag follows them
__global__ void k_copy_words(uint32_t *dst, const uint32_t *src, int32_t nw, uint32_t *tag,
                             uint32_t seq) {
  for (int32_t i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *(volatile uint32_t *)tag = seq;
}

void readback(void *host, const void *dev, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes > (size_t(1) << 20)) {  // bulk copies: straight into the caller's memory
    SA_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    return;
  }
  if (bytes <= 4 * (size_t)kWordsMax && bytes % 4 == 0 && (uintptr_t)dev % 4 == 0) {
    uint32_t *st = (uint32_t *)pinned_buffer(t_words, 4 * (kWordsMax + 1));
    uint32_t *dst = nullptr;
    SA_HIP(hipHostGetDevicePointer((void **)&dst, st, 0));
    // a nonzero tag of this thread's own; the word is cleared first, so a tag left by an
    // earlier readback (or an earlier owner of the buffer) is never taken for this one
    static thread_local uint32_t seq = 0;
    seq = seq + 1 == 0 ? 1 : seq + 1;
    volatile uint32_t *tag = st + kWordsMax;
    *tag = 0;
    k_copy_words<<<1, kBlock, 0, s>>>(dst, (const uint32_t *)dev, (int32_t)(bytes / 4),
                                      dst + kWordsMax, seq);
    SA_LAUNCH_CHECK();
    // wait at most SAAMG_STATUS_SPIN_NS (default 20 ms; 0: synchronise at once), then
    // synchronise the stream, which also reports an earlier kernel's failure
    int64_t spin_ns = 20000000;
    if (const char *e = std::getenv("SAAMG_STATUS_SPIN_NS")) spin_ns = std::atoll(e);
    bool seen = false;
    if (spin_ns > 0) {
      const auto t0 = std::chrono::steady_clock::now();
      for (uint32_t polls = 0;; ++polls) {
        if (*tag == seq) {
          seen = true;
          break;
        }
        if ((polls & 255u) == 255u &&
            std::chrono::duration_cast<std::chrono::nanoseconds>(
                std::chrono::steady_clock::now() - t0)
                    .count() >= spin_ns)
          break;
      }
    }
    if (!seen) SA_HIP(hipStreamSynchronize(s));
    std::atomic_thread_fence(std::memory_order_acquire);
    std::memcpy(host, st, bytes);
    return;
  }
  void *st = pinned_staging(bytes);
  SA_HIP(hipMemcpyAsync(st, dev, bytes, hipMemcpyDeviceToHost, s));
  SA_HIP(hipStreamSynchronize(s));
  std::memcpy(host, st, bytes);
}

}  // namespace sa
