// Instantiation unit: f64 mode products (templates in mode_common.hpp).
// FP64: no register prefetch, two workgroups per CU (measured fastest at 256^3: the
// second workgroup hides the first one's load latency better than a prefetch buffer that
// halves occupancy).
#include "mode_common.hpp"

namespace helm {

// Free-dimension 16-blocks per wave: the table's NB, or 2 or 1 when the table's would leave
// the chip with fewer than two workgroups per CU (small grids, few right-hand sides).  Fewer
// blocks per wave read the eigenvector fragments more often per flop, so the widest choice that
// still fills the chip wins.
constexpr long long kFillBlocks = 512;
inline int narrow_nb(int nb_table, int wn, long long free16) {
  for (int nb : {nb_table, 2, 1}) {
    if (nb > nb_table) continue;
    if ((free16 + wn * nb - 1) / (wn * nb) >= kFillBlocks) return nb;
  }
  return 1;
}
template <typename F>
hipError_t with_nb(int nb_table, int nb, F&& f) {
  if (nb == nb_table) return f(std::integral_constant<int, 0>{});
  if (nb == 2) return f(std::integral_constant<int, 2>{});
  return f(std::integral_constant<int, 1>{});
}

hipError_t mode_left_f64(int ci, const void* Msw, int K, const void* X, void* Y, long long S, long long Nn, Epi epi,
                          const EpiArgs& ep, hipStream_t st) {
  using TC = double;
  const int KB = (K + kblock(P_F64) - 1) / kblock(P_F64);
  if (epi != EPI_STORE && epi != EPI_DIVIDE) return hipErrorInvalidValue;
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int WN = 4 / c.W;
    int nb = narrow_nb(c.NB, WN, (S * Nn + 15) / 16);
    while (nb > 1 && !group_tiles_ok(ep, static_cast<long long>(WN) * nb * 16)) nb = nb > 2 ? 2 : 1;
    if (!group_tiles_ok(ep, static_cast<long long>(WN) * nb * 16)) return hipErrorInvalidValue;
    return with_nb(c.NB, nb, [&](auto nbc) -> hipError_t {
      constexpr int NB = decltype(nbc)::value == 0 ? c.NB : decltype(nbc)::value;
      constexpr int NT = WN * NB * 16;
      const long long blocks = (S * Nn + NT - 1) / NT;
      if (blocks <= 0) return hipSuccess;
      const TC* Mp = static_cast<const TC*>(Msw);
      const TC* Xp = static_cast<const TC*>(X);
      TC* Yp = static_cast<TC*>(Y);
      if (epi == EPI_STORE)
        hipLaunchKernelGGL((k_left<double, c.W, c.MB, NB, EPI_STORE, 2, false>), grid1d(blocks), dim3(256), 0, st, Mp,
                           KB, K, Xp, Yp, S, Nn, ep);
      else
        hipLaunchKernelGGL((k_left<double, c.W, c.MB, NB, EPI_DIVIDE, 2, false>), grid1d(blocks), dim3(256), 0, st, Mp,
                           KB, K, Xp, Yp, S, Nn, ep);
      return hipGetLastError();
    });
  });
}

hipError_t mode_right_f64(int ci, const void* Msw, int K, const void* X, void* Y, long long Mrows, Epi epi, bool vec,
                          const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 15) / 16;
  if (epi != EPI_STORE) return hipErrorInvalidValue;
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int WM = 4 / c.W;
    int nb = narrow_nb(c.NB, WM, (Mrows + 15) / 16);
    while (nb > 1 && !group_tiles_ok(ep, static_cast<long long>(WM) * nb * 16)) nb = nb > 2 ? 2 : 1;
    if (!group_tiles_ok(ep, static_cast<long long>(WM) * nb * 16)) return hipErrorInvalidValue;
    return with_nb(c.NB, nb, [&](auto nbc) -> hipError_t {
      constexpr int RB = decltype(nbc)::value == 0 ? c.NB : decltype(nbc)::value;  // row blocks per wave
      constexpr int MT = WM * RB * 16;
      const long long blocks = (Mrows + MT - 1) / MT;
      if (blocks <= 0) return hipSuccess;
      const double* Mp = static_cast<const double*>(Msw);
      const double* Xp = static_cast<const double*>(X);
      double* Yp = static_cast<double*>(Y);
      if (vec)
        hipLaunchKernelGGL((k_right<double, double, c.W, c.MB, RB, EPI_STORE, true, 2, false>), grid1d(blocks),
                           dim3(256), 0, st, Mp, KB, K, Xp, Yp, Mrows, ep);
      else
        hipLaunchKernelGGL((k_right<double, double, c.W, c.MB, RB, EPI_STORE, false, 2, false>), grid1d(blocks),
                           dim3(256), 0, st, Mp, KB, K, Xp, Yp, Mrows, ep);
      return hipGetLastError();
    });
  });
}

}  // namespace helm
