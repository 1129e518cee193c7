// Caching device allocator behind DevBuf.
//
// A freed block is handed out again only to the host thread that freed it.
// Blocks go back to the cache when their owner is destroyed, which may be
// before the work queued on the owner's stream has run; each thread orders
// its work on its own stream, so reuse within the thread is ordered after
// that work, but another thread's stream would not wait for it (the serving
// loop runs a worker and an assembler thread, each with its own stream).
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

#include "hm_internal.hpp"

namespace hm {

namespace {

struct Pool {
  std::mutex mu;
  // (device, freeing thread, size class) -> block
  std::multimap<std::tuple<int, std::thread::id, size_t>, void*> free_;
  std::map<void*, int> owner;  // block -> device
  int64_t cached = 0;
};

Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: blocks may be released during exit
  return *p;
}

// Size classes: four per power of two above 64 KiB, 256-byte granules below.
size_t size_class(size_t b) {
  if (b <= (64u << 10)) return (b + 255) & ~size_t(255);
  int e = 63 - __builtin_clzll(b);
  size_t step = size_t(1) << (e - 2);
  return (b + step - 1) & ~(step - 1);
}

}  // namespace

void* pool_alloc(size_t bytes, size_t* granted) {
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  const size_t g = size_class(bytes);
  Pool& P = pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.free_.find(std::make_tuple(dev, std::this_thread::get_id(), g));
    if (it != P.free_.end()) {
      void* p = it->second;
      P.free_.erase(it);
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
    P.owner[p] = dev;
  }
  *granted = g;
  return p;
}

void pool_free(void* p, size_t granted) {
  Pool& P = pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = P.owner.find(p);
  const int dev = it != P.owner.end() ? it->second : 0;
  P.free_.emplace(std::make_tuple(dev, std::this_thread::get_id(), granted), p);
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
    (void)hipSetDevice(std::get<0>(kv.first));
    (void)hipDeviceSynchronize();
    (void)hipFree(kv.second);
    P.owner.erase(kv.second);
  }
  (void)hipSetDevice(cur);
  P.free_.clear();
  P.cached = 0;
}

}  // namespace hm
