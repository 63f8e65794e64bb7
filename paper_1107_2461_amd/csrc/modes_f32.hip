// Instantiation unit: f32 mode products (templates in mode_common.hpp).
#include "mode_common.hpp"

namespace helm {

hipError_t mode_left_f32(int ci, const void* Msw, int K, const void* X, void* Y, long long S, long long Nn, Epi epi,
                          const EpiArgs& ep, hipStream_t st) {
  using TC = float;
  const int KB = (K + kblock(P_F32) - 1) / kblock(P_F32);
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr int NT = (4 / kCfgs[CI].W) * kCfgs[CI].NB * 16;
    const long long blocks = (S * Nn + NT - 1) / NT;
    if (blocks <= 0) return hipSuccess;
    const TC* Mp = static_cast<const TC*>(Msw);
    const TC* Xp = static_cast<const TC*>(X);
    TC* Yp = static_cast<TC*>(Y);
    if (epi == EPI_STORE) {
      constexpr int E = EPI_STORE;
      hipLaunchKernelGGL((k_left<float, kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else if (epi == EPI_DIVIDE) {
      constexpr int E = EPI_DIVIDE;
      hipLaunchKernelGGL((k_left<float, kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t mode_right_f32(int ci, const void* Msw, int K, const void* X, void* Y, long long Mrows, Epi epi, bool vec,
                          const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 15) / 16;
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int MT = (4 / c.W) * c.NB * 16;
    const long long blocks = (Mrows + MT - 1) / MT;
    if (blocks <= 0) return hipSuccess;
    const float* Mp = static_cast<const float*>(Msw);
    const float* Xp = static_cast<const float*>(X);
    if (epi == EPI_STORE) {
      float* Yp = static_cast<float*>(Y);
      if (vec)
        hipLaunchKernelGGL((k_right<float, float, c.W, c.MB, c.NB, EPI_STORE, true>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
      else
        hipLaunchKernelGGL((k_right<float, float, c.W, c.MB, c.NB, EPI_STORE, false>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
    } else if (epi == EPI_ACCUM) {
      double* Yp = static_cast<double*>(Y);
      if (vec)
        hipLaunchKernelGGL((k_right<float, double, c.W, c.MB, c.NB, EPI_ACCUM, true>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
      else
        hipLaunchKernelGGL((k_right<float, double, c.W, c.MB, c.NB, EPI_ACCUM, false>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

}  // namespace helm
