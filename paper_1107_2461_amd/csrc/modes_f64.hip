// Instantiation unit: f64 mode products (templates in mode_common.hpp).
// FP64: no register prefetch, two workgroups per CU (measured fastest at 256^3: the
// second workgroup hides the first one's load latency better than a prefetch buffer that
// halves occupancy).
#include "mode_common.hpp"

namespace helm {

hipError_t mode_left_f64(int ci, const void* Msw, int K, const void* X, void* Y, long long S, long long Nn, Epi epi,
                          const EpiArgs& ep, hipStream_t st) {
  using TC = double;
  const int KB = (K + kblock(P_F64) - 1) / kblock(P_F64);
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
      hipLaunchKernelGGL((k_left<double, kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E, 2, false>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else if (epi == EPI_DIVIDE) {
      constexpr int E = EPI_DIVIDE;
      hipLaunchKernelGGL((k_left<double, kCfgs[CI].W, kCfgs[CI].MB, kCfgs[CI].NB, E, 2, false>), grid1d(blocks), dim3(256), 0, st, Mp, KB, K, Xp, Yp, S, Nn, ep);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t mode_right_f64(int ci, const void* Msw, int K, const void* X, void* Y, long long Mrows, Epi epi, bool vec,
                          const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 15) / 16;
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int MT = (4 / c.W) * c.NB * 16;
    const long long blocks = (Mrows + MT - 1) / MT;
    if (blocks <= 0) return hipSuccess;
    const double* Mp = static_cast<const double*>(Msw);
    const double* Xp = static_cast<const double*>(X);
    double* Yp = static_cast<double*>(Y);
    if (epi != EPI_STORE) return hipErrorInvalidValue;
    if (vec)
      hipLaunchKernelGGL((k_right<double, double, c.W, c.MB, c.NB, EPI_STORE, true, 2, false>), grid1d(blocks), dim3(256), 0,
                         st, Mp, KB, K, Xp, Yp, Mrows, ep);
    else
      hipLaunchKernelGGL((k_right<double, double, c.W, c.MB, c.NB, EPI_STORE, false, 2, false>), grid1d(blocks), dim3(256), 0,
                         st, Mp, KB, K, Xp, Yp, Mrows, ep);
    return hipGetLastError();
  });
}

}  // namespace helm
