// Instantiation unit: split-BF16 mode products with rotating layout (rot_bf16x3.hpp).
#include "rot_bf16x3.hpp"

namespace helm {

namespace {

// One launch with RW row blocks per wave.
template <int CI, int RW>
hipError_t launch_rot(const bf16_t* Mp, long long piece, int KB, int K, const void* Xv, bool x_f64, void* Y,
                      long long R, long long PQ, Epi epi, bool vec, const EpiArgs& ep, hipStream_t st) {
  constexpr Cfg c = kCfgs[CI];
  constexpr int MT = (4 / c.W) * RW * 16;
  const long long blocks = (R * PQ + MT - 1) / MT;
  if (blocks <= 0) return hipSuccess;
  auto go = [&](auto epi_c, auto vec_c, auto in_t) {
    using TIn = decltype(in_t);
    hipLaunchKernelGGL((k_rot_bf16x3<c.W, c.MB, RW, decltype(epi_c)::value, decltype(vec_c)::value, TIn>),
                       grid1d(blocks), dim3(256), 0, st, Mp, piece, KB, K, static_cast<const TIn*>(Xv), Y, R, PQ, ep);
  };
  using VT = std::true_type;
  using VF = std::false_type;
  using ES = std::integral_constant<int, EPI_STORE>;
  using ED = std::integral_constant<int, EPI_DIVIDE>;
  using E8 = std::integral_constant<int, EPI_STORE_F64>;
  if (x_f64) {  // first product of a solve: FP64 right-hand side, plain store
    if (epi != EPI_STORE) return hipErrorInvalidValue;
    vec ? go(ES{}, VT{}, double{}) : go(ES{}, VF{}, double{});
  } else if (epi == EPI_STORE) {
    vec ? go(ES{}, VT{}, float{}) : go(ES{}, VF{}, float{});
  } else if (epi == EPI_DIVIDE) {
    vec ? go(ED{}, VT{}, float{}) : go(ED{}, VF{}, float{});
  } else if (epi == EPI_STORE_F64) {
    vec ? go(E8{}, VT{}, float{}) : go(E8{}, VF{}, float{});
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Halves the tile height (row blocks per wave) while a launch would not fill one round of the
// chip (256 CUs x 2 resident workgroups), down to one 16-row block per wave: small grids and
// slabs get enough workgroups, large ones keep the tile that reads M once per 128 rows.
template <int CI, int RW>
hipError_t launch_fit(const bf16_t* Mp, long long piece, int KB, int K, const void* Xv, bool x_f64, void* Y,
                      long long R, long long PQ, Epi epi, bool vec, const EpiArgs& ep, hipStream_t st) {
  constexpr Cfg c = kCfgs[CI];
  constexpr int MT = (4 / c.W) * RW * 16;
  if constexpr (RW > 1) {
    // (a grouped solve also halves it until a tile lies inside one RHS)
    if ((R * PQ + MT - 1) / MT < 512 || !group_tiles_ok(ep, MT))
      return launch_fit<CI, RW / 2>(Mp, piece, KB, K, Xv, x_f64, Y, R, PQ, epi, vec, ep, st);
  }
  if (!group_tiles_ok(ep, MT)) return hipErrorInvalidValue;
  return launch_rot<CI, RW>(Mp, piece, KB, K, Xv, x_f64, Y, R, PQ, epi, vec, ep, st);
}

}  // namespace

hipError_t mode_rot_bf16x3(int ci, const void* Msw, long long piece, int K, const void* Xv, bool x_f64, void* Y,
                           long long R, long long PQ, Epi epi, bool vec, const EpiArgs& ep, hipStream_t st) {
  const int KB = (K + 31) / 32;
  const bf16_t* Mp = static_cast<const bf16_t*>(Msw);
  return for_cfg(ci, [&](auto cic) -> hipError_t {
    constexpr int CI = decltype(cic)::value;
    constexpr Cfg c = kCfgs[CI];
    constexpr int RW = rot_rows(c);  // row blocks per wave of the full tile
    return launch_fit<CI, RW>(Mp, piece, KB, K, Xv, x_f64, Y, R, PQ, epi, vec, ep, st);
  });
}

}  // namespace helm
