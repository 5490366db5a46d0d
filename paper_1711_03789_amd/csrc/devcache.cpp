// Cache of large device blocks (see objects.hpp).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "objects.hpp"

namespace mx {
namespace {

struct Block {
  void *p;
  size_t cap;
  int device;
  hipEvent_t done;  // recorded on the releasing stream; the block is reusable once it completed
};

std::mutex g_mu;
std::vector<Block> g_free;

void drop(Block &b) {
  (void)hipEventSynchronize(b.done);
  (void)hipEventDestroy(b.done);
  (void)hipFree(b.p);
}

}  // namespace

void *big_alloc(size_t n, size_t *capacity) {
  int dev = 0;
  MX_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1;
    // best fit, but never more than 1.5x the request: a small request must not pin a block that a
    // later large one needs (it then gets fresh memory, emptying the cache first if need be)
    for (int i = 0; i < (int)g_free.size(); ++i)
      if (g_free[i].device == dev && g_free[i].cap >= n && g_free[i].cap - n <= n / 2 &&
          (best < 0 || g_free[i].cap < g_free[best].cap))
        best = i;
    if (best >= 0) {
      Block b = g_free[best];
      g_free.erase(g_free.begin() + best);
      MX_HIP(hipEventSynchronize(b.done));
      MX_HIP(hipEventDestroy(b.done));
      *capacity = b.cap;
      return b.p;
    }
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    big_trim(dev);
    e = hipMalloc(&p, n);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? MX_ENOMEM : MX_EDEVICE,
         std::string("hipMalloc of a large block: ") + hipGetErrorString(e));
  }
  *capacity = n;
  return p;
}

void big_free(void *p, size_t capacity, hipStream_t st) {
  int dev = 0;
  hipEvent_t ev = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, st) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
    (void)hipGetLastError();  // leave no error behind for a later launch check
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_free.push_back({p, capacity, dev, ev});
}

size_t big_cached(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  size_t n = 0;
  for (const auto &b : g_free)
    if (b.device == device) n += b.cap;
  return n;
}

void big_trim(int device) {
  std::vector<Block> out;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<Block> keep;
    for (auto &b : g_free) (b.device == device ? out : keep).push_back(b);
    g_free.swap(keep);
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  for (auto &b : out) drop(b);
  (void)hipSetDevice(cur);
}

}  // namespace mx
