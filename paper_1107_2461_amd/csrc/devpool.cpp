// Pool of small device blocks (see alloc.hpp).
#include <hip/hip_runtime_api.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "alloc.hpp"

namespace helm {
namespace {

constexpr size_t kChunk = size_t(32) << 20;  // device memory taken from hipMalloc at a time
constexpr int kClasses = 15;                 // 256 B .. 4 MiB, powers of two

int size_class(size_t bytes) {
  int c = 0;
  size_t s = 256;
  while (s < bytes) {
    s <<= 1;
    ++c;
  }
  return c;
}

struct DevicePool {
  std::vector<char*> free_[kClasses];
  char* cur = nullptr;  // carve position in the newest chunk
  size_t left = 0;
};

std::mutex g_pool_mu;
std::map<int, DevicePool> g_pools;          // by device ordinal; chunks are never returned
struct Owner {
  int device;  // the device the block was taken on
  int cls;     // its size class
};
std::unordered_map<void*, Owner> g_owner;

}  // namespace

hipError_t pool_get(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const int c = size_class(bytes);
  const size_t sz = size_t(256) << c;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  DevicePool& dp = g_pools[dev];
  if (!dp.free_[c].empty()) {
    *p = dp.free_[c].back();
    dp.free_[c].pop_back();
    g_owner[*p] = Owner{dev, c};
    return hipSuccess;
  }
  if (dp.left < sz) {
    void* chunk = nullptr;
    if ((e = hipMalloc(&chunk, kChunk)) != hipSuccess) return e;
    // the rest of the old chunk is handed out as blocks of its largest classes
    while (dp.left >= 256) {
      int k = size_class(dp.left);
      if ((size_t(256) << k) > dp.left) --k;
      dp.free_[k].push_back(dp.cur);
      dp.cur += size_t(256) << k;
      dp.left -= size_t(256) << k;
    }
    dp.cur = static_cast<char*>(chunk);
    dp.left = kChunk;
  }
  *p = dp.cur;
  dp.cur += sz;
  dp.left -= sz;
  g_owner[*p] = Owner{dev, c};
  return hipSuccess;
}

void pool_put(void* p, size_t) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_owner.find(p);
  if (it == g_owner.end()) return;  // not a pool block
  // the block goes back under the class it was taken with, whatever size the caller names
  g_pools[it->second.device].free_[it->second.cls].push_back(static_cast<char*>(p));
  g_owner.erase(it);
}

}  // namespace helm
