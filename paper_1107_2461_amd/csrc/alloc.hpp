// Device allocation through the caller's optional allocator callback (helm_opts.alloc), else
// hipMalloc / hipFree.  Every object that allocates device memory keeps the DevAlloc it was
// built with and releases through it.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/helm.h"

namespace helm {

// Blocks of at most kPoolMax bytes without a caller's allocator come from a per-device pool
// (devpool.cpp): 32 MiB chunks from hipMalloc, kept until the process ends, carved into
// power-of-two blocks that are recycled through free lists.  hipFree synchronizes the whole
// device, so freeing a plan's tables directly would make a thread that releases a plan while
// other solves run (the solve server evicting a resident plan) wait for all of them.  A block
// is taken on the current device and goes back to that device's pool whichever is current.
constexpr size_t kPoolMax = size_t(4) << 20;
hipError_t pool_get(void** p, size_t bytes);
void pool_put(void* p, size_t bytes);

struct DevAlloc {
  helm_alloc_fn alloc = nullptr;
  helm_free_fn dealloc = nullptr;
  void* ctx = nullptr;

  static DevAlloc from(const helm_opts& o) { return DevAlloc{o.alloc, o.dealloc, o.alloc_ctx}; }
  bool valid() const { return (alloc == nullptr) == (dealloc == nullptr); }

  hipError_t get(void** p, size_t bytes) const {
    if (bytes == 0) bytes = 1;
    if (!alloc) return bytes <= kPoolMax ? pool_get(p, bytes) : hipMalloc(p, bytes);
    *p = alloc(bytes, ctx);
    if (!*p) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(*p) % 256 != 0) {  // the kernels assume 256-byte alignment
      dealloc(*p, bytes, ctx);
      *p = nullptr;
      return hipErrorInvalidValue;
    }
    return hipSuccess;
  }
  void put(void* p, size_t bytes) const {
    if (!p) return;
    if (bytes == 0) bytes = 1;
    if (!dealloc) {
      if (bytes <= kPoolMax)
        pool_put(p, bytes);
      else
        (void)hipFree(p);
      return;
    }
    dealloc(p, bytes, ctx);
  }
  // Identity of the allocator, for cache keys: objects built with different allocators are
  // never shared.
  std::string key() const {
    std::string k;
    const void* ids[3] = {reinterpret_cast<const void*>(alloc), reinterpret_cast<const void*>(dealloc), ctx};
    k.append(reinterpret_cast<const char*>(ids), sizeof(ids));
    return k;
  }
};

}  // namespace helm
