// Instantiation unit: split-BF16 mode products with rotating layout (rot_bf16x3.hpp).
#include "rot_bf16x3.hpp"

namespace helm {

hipError_t mode_rot_bf16x3(int ci, const void* Msw, long long piece, int K, const void* Xv, bool x_f64, void* Y,
                           long long R, long long PQ, Epi epi, bool vec, const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 31) / 32;
  const bf16_t* Mp = static_cast<const bf16_t*>(Msw);
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int RW = rot_rows(c);             // row blocks per wave
    constexpr int MT = (4 / c.W) * RW * 16;
    const long long blocks = (R * PQ + MT - 1) / MT;
    if (blocks <= 0) return hipSuccess;
    const float* X = static_cast<const float*>(Xv);
#define HELM_ROT(E)                                                                                               \
  do {                                                                                                            \
    if (vec)                                                                                                      \
      hipLaunchKernelGGL((k_rot_bf16x3<c.W, c.MB, RW, E, true>), grid1d(blocks), dim3(256), 0, st, Mp, piece, KB, \
                         K, X, Y, R, PQ, ep);                                                                     \
    else                                                                                                          \
      hipLaunchKernelGGL((k_rot_bf16x3<c.W, c.MB, RW, E, false>), grid1d(blocks), dim3(256), 0, st, Mp, piece,   \
                         KB, K, X, Y, R, PQ, ep);                                                                 \
  } while (0)
    if (x_f64) {  // first product of a solve: FP64 right-hand side, plain store
      if (epi != EPI_STORE) return hipErrorInvalidValue;
      const double* Xd = static_cast<const double*>(Xv);
      if (vec)
        hipLaunchKernelGGL((k_rot_bf16x3<c.W, c.MB, RW, EPI_STORE, true, double>), grid1d(blocks), dim3(256), 0, st,
                           Mp, piece, KB, K, Xd, Y, R, PQ, ep);
      else
        hipLaunchKernelGGL((k_rot_bf16x3<c.W, c.MB, RW, EPI_STORE, false, double>), grid1d(blocks), dim3(256), 0,
                           st, Mp, piece, KB, K, Xd, Y, R, PQ, ep);
      return hipGetLastError();
    }
    if (epi == EPI_STORE)
      HELM_ROT(EPI_STORE);
    else if (epi == EPI_DIVIDE)
      HELM_ROT(EPI_DIVIDE);
    else if (epi == EPI_STORE_F64)
      HELM_ROT(EPI_STORE_F64);
    else
      return hipErrorInvalidValue;
#undef HELM_ROT
    return hipGetLastError();
  });
}

}  // namespace helm
