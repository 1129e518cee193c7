// Caching device allocator behind DevBuf, with stream-ordered reuse.
//
// A block goes back to the cache when its owner is destroyed, which may be
// before the work queued on the owner's stream has run.  The freeing thread's
// current stream (set by the entry points, see StreamScope) is remembered
// with the block, and an event is recorded on it.  A later allocation on the
// same stream takes the block at once (its work is ordered after the earlier
// work); an allocation on any other stream makes that stream wait for the
// event first, so no stream can reuse a block that kernels queued on another
// stream may still read or write.  Blocks freed while their stream is being
// captured into a graph get no event and are reused on that stream only.
#include <map>
#include <mutex>
#include <tuple>

#include "hm_internal.hpp"

namespace hm {

namespace {

struct FreeBlock {
  void* p;
  hipStream_t s;  // the stream the block was freed on
  bool ev_ok;     // the block's event marks the end of its work on s
};

struct BlockInfo {
  int dev = 0;
  hipEvent_t ev = nullptr;
};

struct Pool {
  std::mutex mu;
  // (device, size class) -> free blocks
  std::multimap<std::pair<int, size_t>, FreeBlock> free_;
  std::map<void*, BlockInfo> info;  // every block the pool has allocated
  int64_t cached = 0;
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: blocks may be released during exit
  return *p;
}

thread_local hipStream_t tl_stream = nullptr;

// Size classes: four per power of two above 64 KiB, 256-byte granules below.
size_t size_class(size_t b) {
  if (b <= (64u << 10)) return (b + 255) & ~size_t(255);
  int e = 63 - __builtin_clzll(b);
  size_t step = size_t(1) << (e - 2);
  return (b + step - 1) & ~(step - 1);
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // unknown: treat as capturing (same-stream reuse only)
  }
  return cs != hipStreamCaptureStatusNone;
}

}  // namespace

hipStream_t current_stream() { return tl_stream; }
void set_current_stream(hipStream_t s) { tl_stream = s; }

void* pool_alloc(size_t bytes, size_t* granted) {
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  const size_t g = size_class(bytes);
  const hipStream_t cur = tl_stream;
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto range = P.free_.equal_range(std::make_pair(dev, g));
    auto pick = P.free_.end();
    for (auto it = range.first; it != range.second; ++it)
      if (it->second.s == cur) {
        pick = it;
        break;
      }
    if (pick == P.free_.end() && range.first != range.second && !capturing(cur)) {
      for (auto it = range.first; it != range.second; ++it)
        if (it->second.ev_ok) {
          hipEvent_t ev = P.info[it->second.p].ev;
          if (hipStreamWaitEvent(cur, ev, 0) == hipSuccess) {
            pick = it;
            break;
          }
          (void)hipGetLastError();
        }
    }
    if (pick != P.free_.end()) {
      void* p = pick->second.p;
      P.free_.erase(pick);
      P.cached -= (int64_t)g;
      *granted = g;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, g);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    pool_trim();
    e = hipMalloc(&p, g);
  }
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? HM_ENOMEM : HM_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(P.mu);
    P.info[p].dev = dev;
  }
  *granted = g;
  return p;
}

void pool_free(void* p, size_t granted) {
  Pool& P = pool();
  const hipStream_t s = tl_stream;
  std::lock_guard<std::mutex> lk(P.mu);
  BlockInfo& bi = P.info[p];
  bool ev_ok = false;
  if (!capturing(s)) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != bi.dev) (void)hipSetDevice(bi.dev);
    if (!bi.ev && hipEventCreateWithFlags(&bi.ev, hipEventDisableTiming) != hipSuccess) bi.ev = nullptr;
    ev_ok = bi.ev && hipEventRecord(bi.ev, s) == hipSuccess;
    (void)hipGetLastError();
    if (cur != bi.dev) (void)hipSetDevice(cur);
  }
  P.free_.emplace(std::make_pair(bi.dev, granted), FreeBlock{p, s, ev_ok});
  P.cached += (int64_t)granted;
}

int64_t pool_cached_bytes() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  return P.cached;
}

void pool_trim() {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : P.free_) {
    (void)hipSetDevice(kv.first.first);
    (void)hipDeviceSynchronize();
    (void)hipFree(kv.second.p);
    auto it = P.info.find(kv.second.p);
    if (it != P.info.end()) {
      if (it->second.ev) (void)hipEventDestroy(it->second.ev);
      P.info.erase(it);
    }
  }
  (void)hipSetDevice(cur);
  P.free_.clear();
  P.cached = 0;
}

}  // namespace hm
