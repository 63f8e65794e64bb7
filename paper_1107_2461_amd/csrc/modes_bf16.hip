// Instantiation unit: bf16 mode products (templates in mode_common.hpp).
#include "mode_common.hpp"

namespace helm {

hipError_t mode_left_bf16(int ci, const void* Msw, int K, const void* X, void* Y, long long S, long long Nn, Epi epi,
                          const EpiArgs& ep, hipStream_t st) {
  using TC = bf16_t;
  const int KB = (K + kblock(P_BF16) - 1) / kblock(P_BF16);
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
      hipLaunchKernelGGL((k_left_bf16<kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else if (epi == EPI_DIVIDE) {
      constexpr int E = EPI_DIVIDE;
      hipLaunchKernelGGL((k_left_bf16<kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t mode_right_bf16(int ci, const void* Msw, int K, const void* X, void* Y, long long Mrows, Epi epi, bool vec,
                           const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 31) / 32;
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int MT = (4 / c.W) * c.NB * 16;
    const long long blocks = (Mrows + MT - 1) / MT;
    if (blocks <= 0) return hipSuccess;
    const bf16_t* Mp = static_cast<const bf16_t*>(Msw);
    const bf16_t* Xp = static_cast<const bf16_t*>(X);
    if (epi == EPI_STORE) {
      bf16_t* Yp = static_cast<bf16_t*>(Y);
      if (vec)
        hipLaunchKernelGGL((k_right_bf16<bf16_t, c.W, c.MB, c.NB, EPI_STORE, true>), grid1d(blocks), dim3(256), 0, st,
                           Mp, KB, K, Xp, Yp, Mrows, ep);
      else
        hipLaunchKernelGGL((k_right_bf16<bf16_t, c.W, c.MB, c.NB, EPI_STORE, false>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
    } else if (epi == EPI_ACCUM) {
      double* Yp = static_cast<double*>(Y);
      if (vec)
        hipLaunchKernelGGL((k_right_bf16<double, c.W, c.MB, c.NB, EPI_ACCUM, true>), grid1d(blocks), dim3(256), 0, st,
                           Mp, KB, K, Xp, Yp, Mrows, ep);
      else
        hipLaunchKernelGGL((k_right_bf16<double, c.W, c.MB, c.NB, EPI_ACCUM, false>), grid1d(blocks), dim3(256), 0,
                           st, Mp, KB, K, Xp, Yp, Mrows, ep);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

}  // namespace helm
