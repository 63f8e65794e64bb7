// Measurement probes (no solve calls them): loops of independent MFMAs on register operands
// and a streaming copy.  They give the matrix rate per precision and the HBM rate that the
// chip sustains on this software stack, beside the datasheet peaks that the kernel rooflines
// are quoted against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/helm.h"
#include "mode_common.hpp"

namespace helm {
namespace {

// KIND 0: BF16 16x16x32 (FP32 accumulation), 1: FP32 16x16x4, 2: FP64 16x16x4; kChains
// independent accumulators per wave (the best count differs between the forms).
template <int KIND, int kChains>
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  float s = 0.f;
  if constexpr (KIND == 0) {
    u16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {  // bfloat16 values in [1, 2): 0x3f80 plus a small mantissa
      a[j] = static_cast<unsigned short>(0x3f80 + ((lane + j) & 15));
      b[j] = static_cast<unsigned short>(0x3f80 + ((lane * 3 + j) & 15));
    }
    f4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = mma_bf16(a, b, acc[c]);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else if constexpr (KIND == 1) {
    const float a = 1.f + lane * 1e-3f, b = 1.f - lane * 1e-3f;
    f4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = Mma<float>::mma(a, b, acc[c]);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else {
    const double a = 1.0 + lane * 1e-3, b = 1.0 - lane * 1e-3;
    d4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = d4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = Mma<double>::mma(a, b, acc[c]);
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    s = static_cast<float>(t);
  }
  out[static_cast<long long>(blockIdx.x) * 256 + threadIdx.x] = s;  // keeps the chains live
}

// Each thread moves four 16-byte values, 4 KB apart within its workgroup's 16 KB span, with
// the four loads issued before the first store.
__global__ __launch_bounds__(256) void k_probe_copy(const f4* __restrict__ src, f4* __restrict__ dst, long long n) {
  const long long base = static_cast<long long>(blockIdx.x) * 1024 + threadIdx.x;
  f4 v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (base + q * 256 < n) v[q] = src[base + q * 256];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (base + q * 256 < n) dst[base + q * 256] = v[q];
}

}  // namespace
}  // namespace helm

using namespace helm;

namespace {
template <int KIND>
void launch_probe(int chains, int iters, int blocks, float* out, hipStream_t st) {
  if (chains == 4)
    hipLaunchKernelGGL((k_probe_mfma<KIND, 4>), dim3(blocks), dim3(256), 0, st, iters, out);
  else if (chains == 8)
    hipLaunchKernelGGL((k_probe_mfma<KIND, 8>), dim3(blocks), dim3(256), 0, st, iters, out);
  else
    hipLaunchKernelGGL((k_probe_mfma<KIND, 16>), dim3(blocks), dim3(256), 0, st, iters, out);
}
}  // namespace

extern "C" helm_status helm_probe_mfma(int kind, int chains, int iters, int blocks, float* out, void* stream,
                                       double* flops) {
  if (kind < 0 || kind > 2 || iters < 1 || blocks < 1 || !out) return HELM_EINVAL;
  if (chains != 4 && chains != 8 && chains != 16) return HELM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double per_mfma = kind == 0 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
  if (flops) *flops = per_mfma * chains * static_cast<double>(iters) * blocks * 4;  // four waves per block
  if (kind == 0)
    launch_probe<0>(chains, iters, blocks, out, st);
  else if (kind == 1)
    launch_probe<1>(chains, iters, blocks, out, st);
  else
    launch_probe<2>(chains, iters, blocks, out, st);
  return hipGetLastError() == hipSuccess ? HELM_OK : HELM_EDEVICE;
}

extern "C" helm_status helm_probe_copy(const void* src, void* dst, long long bytes, void* stream) {
  if (!src || !dst || bytes <= 0 || bytes % 16) return HELM_EINVAL;
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) return HELM_EINVAL;
  const char* s = static_cast<const char*>(src);
  const char* d = static_cast<const char*>(dst);
  if (s < d + bytes && d < s + bytes) return HELM_EINVAL;  // overlapping ranges
  const long long n = bytes / 16;
  const long long blocks = (n + 1023) / 1024;
  if (blocks > 0x7fffffffLL) return HELM_EINVAL;
  hipLaunchKernelGGL(k_probe_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const f4*>(src), static_cast<f4*>(dst), n);
  return hipGetLastError() == hipSuccess ? HELM_OK : HELM_EDEVICE;
}
