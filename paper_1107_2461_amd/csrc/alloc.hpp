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

struct DevAlloc {
  helm_alloc_fn alloc = nullptr;
  helm_free_fn dealloc = nullptr;
  void* ctx = nullptr;

  static DevAlloc from(const helm_opts& o) { return DevAlloc{o.alloc, o.dealloc, o.alloc_ctx}; }
  bool valid() const { return (alloc == nullptr) == (dealloc == nullptr); }

  hipError_t get(void** p, size_t bytes) const {
    if (bytes == 0) bytes = 1;
    if (!alloc) return hipMalloc(p, bytes);
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
