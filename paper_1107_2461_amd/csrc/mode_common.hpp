// Mode-product kernels (device templates), included by one instantiation unit per precision.
//
// Each of the six 1D transforms of eq. 29 contracts one axis of the grid function with an
// N x N eigenvector matrix M (E^{-1} forward, E inverse).  With the grid stored x fastest
// this is one of two GEMM shapes:
//   right form (x axis, contiguous):  Y[m][a] = sum_i X[m][i] M[a][i]
//   left form  (y, z axes, strided):  Y[s][a][n] = sum_i M[a][i] X[s][i][n]
// Both run on MFMA 16x16 tiles (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32 with FP32
// accumulation).  A workgroup of 4 waves owns a strip of the output that spans ALL N values
// of the contracted axis, so every element of X is fetched from HBM once and reused N times
// from registers; M (at most 2 MB) is shared by every workgroup and stays in L2.  M is
// swizzled on the host into MFMA fragment order, so one fragment is one coalesced 512-byte
// (1-KB for BF16) read.  Inside each k-block the contraction index is permuted so that
// each lane's values of one operand row are contiguous (one vector load): lane group
// g = lane / 16 at sub-step s covers k = 4g + s (8g + j for BF16).  Both operands use the
// same permutation, so every MFMA still forms the exact inner product.
//
// Epilogues: the pointwise divide of eqs. 26-28 (denominators in FP64) is fused into the
// z-forward product; the refinement update u += du (FP64, with per-RHS max norms) is fused
// into the x-inverse product.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>

#include "kernels.hpp"

namespace helm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t bf16_t;  // storage of a bfloat16 value

// float -> bfloat16, round-to-nearest-even on the 16 discarded bits.
__host__ __device__ inline bf16_t f32_to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<bf16_t>(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

template <typename TOut> __device__ inline TOut store_cvt(double x);
template <> __device__ inline double store_cvt<double>(double x) { return x; }
template <> __device__ inline float store_cvt<float>(double x) { return static_cast<float>(x); }
template <> __device__ inline bf16_t store_cvt<bf16_t>(double x) { return f32_to_bf16(static_cast<float>(x)); }

// Pointers into global memory for data whose pointer is itself loaded from memory (the per-RHS
// tables of a grouped solve): typed in the global address space, so the loads through them are
// global loads.  A generic pointer would give flat loads, which also hold the LDS counter and so
// stall every wait on LDS reads behind them.
template <typename T>
using gptr_t = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr_t<T> to_global(const T* p) {
  return (gptr_t<T>)p;
}
template <typename V, typename T>
__device__ inline V gload(gptr_t<T> p) {
  return *reinterpret_cast<gptr_t<V>>(p);
}
// Entry i of a per-RHS pointer table (read as global memory), or `one` without a table.
template <typename T, typename U>
__device__ inline gptr_t<T> rhs_ptr(const U* const* tab, long long i, const T* one) {
  return tab ? to_global(static_cast<const T*>(to_global(tab)[i])) : to_global(one);
}

// Output layout of the 16x16 MFMA tiles: lane l holds column l % 16; its accumulator
// register r holds row 4 * (l / 16) + r for the FP32 and BF16 forms but row (l / 16) + 4 r
// for the FP64 form (measured on gfx950 with a one-wave probe).
template <typename TC> struct Mma;
template <> struct Mma<double> {
  using acc_t = d4;
  using vec_t = d4;
  static __device__ inline int row(int g, int r) { return g + 4 * r; }
  static __device__ inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<float> {
  using acc_t = f4;
  using vec_t = f4;
  static __device__ inline int row(int g, int r) { return 4 * g + r; }
  static __device__ inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
__device__ inline f4 mma_bf16(u16x8 a, u16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}

// ------------------------------------------------------------------ tile configurations
// (W, MB, NB): W waves span the contracted-axis extent, each with MB 16-row blocks of it;
// the other 4/W waves span the free dimension, each with NB 16-wide blocks.
struct Cfg {
  int W, MB, NB;
};
constexpr Cfg kCfgs[] = {
    {1, 1, 8}, {1, 2, 8}, {1, 4, 4}, {2, 3, 4}, {2, 4, 4}, {2, 5, 3}, {4, 3, 4}, {2, 7, 2}, {4, 4, 4}, {4, 8, 2},
};
constexpr int kNumCfgs = static_cast<int>(sizeof(kCfgs) / sizeof(kCfgs[0]));
constexpr int cfg_extent(Cfg c) { return c.W * c.MB * 16; }

inline int choose_cfg(int K) {
  int best = -1;
  for (int i = 0; i < kNumCfgs; ++i) {
    const int e = cfg_extent(kCfgs[i]);
    if (e < K) continue;
    if (best < 0 || e < cfg_extent(kCfgs[best])) best = i;
  }
  return best;
}
inline int kblock(Prec p) { return p == P_BF16 ? 32 : 16; }

// ------------------------------------------------------------------ epilogue helpers
// Shift of one (x, y) column of the z-forward output: lam_x(a) + lam_y(b) + sigma(r), with
// n = b * nx + a the column inside the RHS r.
__device__ inline double column_shift(const EpiArgs& ep, long long n, int r) {
  const int ni = static_cast<int>(n);
  const int by = ni / ep.nx;
  const gptr_t<double> lx = rhs_ptr(ep.lamx_rhs, r, ep.lamx);
  const gptr_t<double> ly = rhs_ptr(ep.lamy_rhs, r, ep.lamy);
  return lx[ni - by * ep.nx] + ly[by] + ep.sigma[r];
}
// Pointwise divide of eqs. 26-27 with the FP64 denominator lam_z(c) + shift; the exact zero
// denominator of the all-Neumann null mode gives 0 (projection) or v (eq. 28: Lambda := 1).
// FP64 reciprocal: hardware estimate refined by two Newton steps (error a few ulp), which is
// much cheaper than a correctly rounded division inside an MFMA epilogue.
__device__ inline double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double divide_den(double v, const EpiArgs& ep, double den) {
  if (den == 0.0) return ep.eq28 ? v : 0.0;
  return v * recip(den);
}
// The same as a select: an epilogue that divides then has no control-flow joins between its
// stores, where a wait for an earlier load would also wait for every store issued so far.
__device__ inline double divide_den_sel(double v, const EpiArgs& ep, double den) {
  const double q = v * recip(den);
  return den == 0.0 ? (ep.eq28 ? v : 0.0) : q;
}
__device__ inline double divide_by_eigs(double v, const EpiArgs& ep, int c, double shift) {
  return divide_den(v, ep, ep.lamz[c] + shift);
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, static_cast<unsigned long long>(__double_as_longlong(v)));
}
// striped norm slot of quantity q (0: max|du|, 1: max|u|) of RHS r for this workgroup
__device__ inline unsigned long long* norm_slot(unsigned long long* norms, long long r, int q) {
  return norms + (2 * r + q) * kNormStripes + (blockIdx.x % kNormStripes);
}

// RHS index of row m of the x-mode matrix, given the RHS r_lo of the workgroup's first row.
__device__ inline long long rhs_of_row(long long m, long long r_lo, long long rows_per_rhs) {
  long long r = r_lo, b = (r_lo + 1) * rows_per_rhs;
  while (m >= b) {
    ++r;
    b += rows_per_rhs;
  }
  return r;
}

// Per-lane running maxima of |du| and |u| for the two RHS a workgroup can straddle.
struct NormAcc {
  double dmax[2] = {0.0, 0.0}, umax[2] = {0.0, 0.0};
  __device__ inline void add(const EpiArgs& ep, long long r_lo, long long rr, double du, double un) {
    const double ad = fabs(du), au = fabs(un);
    if (!(ad == ad) || !(au == au)) {  // NaN: record it as the largest bit pattern
      atomic_max_nonneg(norm_slot(ep.norms, rr, 0), __longlong_as_double(0x7ff8000000000000ll));
      return;
    }
    if (rr == r_lo) {
      dmax[0] = fmax(dmax[0], ad);
      umax[0] = fmax(umax[0], au);
    } else if (rr == r_lo + 1) {
      dmax[1] = fmax(dmax[1], ad);
      umax[1] = fmax(umax[1], au);
    } else {
      atomic_max_nonneg(norm_slot(ep.norms, rr, 0), ad);
      atomic_max_nonneg(norm_slot(ep.norms, rr, 1), au);
    }
  }
  __device__ inline void flush(const EpiArgs& ep, long long r_lo, long long nrhs, int lane) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double dm = wave_max(dmax[t]), um = wave_max(umax[t]);
      if (lane == 0 && r_lo + t < nrhs) {
        atomic_max_nonneg(norm_slot(ep.norms, r_lo + t, 0), dm);
        atomic_max_nonneg(norm_slot(ep.norms, r_lo + t, 1), um);
      }
    }
  }
};

// ------------------------------------------------------------------ FP64 / FP32 left form
template <typename TC, int W, int MB, int NB, int EPI, int MINB = 1, bool PF = true>
__global__ __launch_bounds__(256, MINB) void k_left(const TC* __restrict__ Msw, int KB, int K,
                                                    const TC* __restrict__ X, TC* __restrict__ Y, long long S,
                                                    long long Nn, EpiArgs ep) {
  using T = Mma<TC>;
  using acc_t = typename T::acc_t;
  using vec_t = typename T::vec_t;
  constexpr int WN = 4 / W;
  constexpr int NT = WN * NB * 16;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % W, wn = wave / W;
  const int l16 = lane & 15, g = lane >> 4;
  const long long total = S * Nn;
  const long long c0 = static_cast<long long>(blockIdx.x) * NT + wn * NB * 16;
  const int rb0 = wm * MB;
  // grouped solve: the workgroup's columns lie inside one RHS, whose plan gives M and lambda_z
  const long long rg = ep.msw_rhs ? static_cast<long long>(blockIdx.x) * NT / ep.span : 0;
  const gptr_t<TC> Mp = rhs_ptr(ep.msw_rhs, rg, Msw);
  [[maybe_unused]] const gptr_t<double> lamz = rhs_ptr(ep.lamz_rhs, rg, ep.lamz);
  // FP64 divide: lambda_z of every output row staged in LDS before the main loop, so the
  // epilogue reads no global memory between its stores (FP32 keeps the registers of kPre below,
  // measured faster there)
  constexpr bool kLds = EPI == EPI_DIVIDE && std::is_same<TC, double>::value;
  constexpr int NLZ = kLds ? W * MB * 16 : 1;
  [[maybe_unused]] __shared__ double sh_lz[NLZ];
  if constexpr (kLds) {
    for (int a = threadIdx.x; a < NLZ; a += blockDim.x) sh_lz[a] = a < K ? lamz[a] : 1.0;
    __syncthreads();
  }

  long long base[NB];
  bool colok[NB];
  [[maybe_unused]] double den_xy[NB];  // lam_x(a) + lam_y(b) + sigma(r) of this lane's columns
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const long long c = c0 + nb * 16 + l16;
    colok[nb] = c < total;
    const long long s = colok[nb] ? c / Nn : 0;
    const long long n = colok[nb] ? c - s * Nn : 0;
    base[nb] = s * K * Nn + n;
    if constexpr (EPI == EPI_DIVIDE) den_xy[nb] = colok[nb] ? column_shift(ep, n, static_cast<int>(s)) : 1.0;
  }
  acc_t acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = acc_t{0, 0, 0, 0};

  vec_t a_cur[MB], a_nxt[MB];
  TC b_cur[NB][4], b_nxt[NB][4];
  auto load = [&](int kb, vec_t(&a)[MB], TC(&b)[NB][4]) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      a[mb] = gload<vec_t>(Mp + ((static_cast<long long>(rb0 + mb) * KB + kb) * 64 + lane) * 4);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = kb * 16 + 4 * g + s;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        b[nb][s] = (colok[nb] && k < K) ? X[base[nb] + static_cast<long long>(k) * Nn] : TC(0);
    }
  };
  if constexpr (PF) load(0, a_cur, b_cur);
  for (int kb = 0; kb < KB; ++kb) {
    if constexpr (PF) {
      if (kb + 1 < KB) load(kb + 1, a_nxt, b_nxt);
    } else {
      load(kb, a_cur, b_cur);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = T::mma(a_cur[mb][s], b_cur[nb][s], acc[mb][nb]);
    if (PF && kb + 1 < KB) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a_cur[mb] = a_nxt[mb];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int s = 0; s < 4; ++s) b_cur[nb][s] = b_nxt[nb][s];
    }
  }
  // divide in the low-precision products: eigenvalues of the lane's rows, all loaded before the first store (the vector-
  // memory counter also counts stores: a load issued after a store would wait for it); the
  // widest entry (NB = 8, K <= 32) has no registers to spare and loads them at the store
  constexpr bool kPre = EPI == EPI_DIVIDE && !kLds && NB <= 4;
  [[maybe_unused]] double lz[kPre ? MB : 1][4];
  if constexpr (kPre) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = (rb0 + mb) * 16 + T::row(g, r);
        lz[mb][r] = a < K ? lamz[a] : 1.0;
      }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = (rb0 + mb) * 16 + T::row(g, r);
        if (a >= K || !colok[nb]) continue;
        const long long idx = base[nb] + static_cast<long long>(a) * Nn;
        if constexpr (EPI == EPI_DIVIDE) {
          if constexpr (kLds) {
            Y[idx] = store_cvt<TC>(divide_den_sel(static_cast<double>(acc[mb][nb][r]), ep, sh_lz[a] + den_xy[nb]));
          } else {
            const double lza = kPre ? lz[kPre ? mb : 0][r] : lamz[a];
            Y[idx] = store_cvt<TC>(divide_den(static_cast<double>(acc[mb][nb][r]), ep, lza + den_xy[nb]));
          }
        } else {
          Y[idx] = static_cast<TC>(acc[mb][nb][r]);
        }
      }
}

// ------------------------------------------------------------------ FP64 / FP32 right form
// Table entry (W, MB, NB) read with roles swapped: W waves span the K output columns with
// NB := MB column blocks each; the 4/W other waves span rows with MB := NB row blocks each.
template <typename TC, typename TOut, int W, int NB, int MB, int EPI, bool VEC, int MINB = 1, bool PF = true>
__global__ __launch_bounds__(256, MINB) void k_right(const TC* __restrict__ Msw, int KB, int K,
                                                     const TC* __restrict__ X, TOut* __restrict__ Y, long long Mrows,
                                                     EpiArgs ep) {
  using T = Mma<TC>;
  using acc_t = typename T::acc_t;
  using vec_t = typename T::vec_t;
  constexpr int WM = 4 / W;
  constexpr int MT = WM * MB * 16;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wn = wave % W, wm = wave / W;
  const int l16 = lane & 15, g = lane >> 4;
  const long long mwg = static_cast<long long>(blockIdx.x) * MT;
  const long long m0 = mwg + wm * MB * 16;
  const int cb0 = wn * NB;
  // grouped solve: the workgroup's rows lie inside one RHS, whose plan gives M
  const gptr_t<TC> Mp = rhs_ptr(ep.msw_rhs, ep.msw_rhs ? mwg / ep.span : 0, Msw);

  const TC* rowp[MB];
  bool rowok[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const long long row = m0 + mb * 16 + l16;
    rowok[mb] = row < Mrows;
    rowp[mb] = X + (rowok[mb] ? row : 0) * K;
  }
  acc_t acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = acc_t{0, 0, 0, 0};

  vec_t a_cur[MB], a_nxt[MB];
  vec_t b_cur[NB], b_nxt[NB];
  auto load = [&](int kb, vec_t(&a)[MB], vec_t(&b)[NB]) {
    const int kq = kb * 16 + 4 * g;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      if constexpr (VEC) {
        a[mb] = (rowok[mb] && kq < K) ? *reinterpret_cast<const vec_t*>(rowp[mb] + kq) : vec_t{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[mb][s] = (rowok[mb] && kq + s < K) ? rowp[mb][kq + s] : TC(0);
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      b[nb] = gload<vec_t>(Mp + ((static_cast<long long>(cb0 + nb) * KB + kb) * 64 + lane) * 4);
  };
  if constexpr (PF) load(0, a_cur, b_cur);
  for (int kb = 0; kb < KB; ++kb) {
    if constexpr (PF) {
      if (kb + 1 < KB) load(kb + 1, a_nxt, b_nxt);
    } else {
      load(kb, a_cur, b_cur);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = T::mma(a_cur[mb][s], b_cur[nb][s], acc[mb][nb]);
    if (PF && kb + 1 < KB) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a_cur[mb] = a_nxt[mb];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b_cur[nb] = b_nxt[nb];
    }
  }
  [[maybe_unused]] NormAcc na;
  [[maybe_unused]] const long long r_lo = (EPI == EPI_ACCUM) ? mwg / ep.rows_per_rhs : 0;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long m = m0 + mb * 16 + T::row(g, r);
      if (m >= Mrows) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int a = (cb0 + nb) * 16 + l16;
        if (a >= K) continue;
        const long long idx = m * K + a;
        if constexpr (EPI == EPI_ACCUM) {
          const double du = static_cast<double>(acc[mb][nb][r]);
          const double un = (ep.accum_zero ? 0.0 : static_cast<double>(Y[idx])) + du;
          Y[idx] = store_cvt<TOut>(un);
          na.add(ep, r_lo, rhs_of_row(m, r_lo, ep.rows_per_rhs), du, un);
        } else {
          Y[idx] = store_cvt<TOut>(static_cast<double>(acc[mb][nb][r]));
        }
      }
    }
  if constexpr (EPI == EPI_ACCUM) na.flush(ep, r_lo, (Mrows + ep.rows_per_rhs - 1) / ep.rows_per_rhs, lane);
}

// ------------------------------------------------------------------ BF16 left form
template <int W, int MB, int NB, int EPI>
__global__ __launch_bounds__(256) void k_left_bf16(const bf16_t* __restrict__ Msw, int KB, int K,
                                                   const bf16_t* __restrict__ X, bf16_t* __restrict__ Y, long long S,
                                                   long long Nn, EpiArgs ep) {
  constexpr int WN = 4 / W;
  constexpr int NT = WN * NB * 16;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % W, wn = wave / W;
  const int l16 = lane & 15, g = lane >> 4;
  const long long total = S * Nn;
  const long long c0 = static_cast<long long>(blockIdx.x) * NT + wn * NB * 16;
  const int rb0 = wm * MB;
  long long base[NB];
  bool colok[NB];
  [[maybe_unused]] double den_xy[NB];  // lam_x(a) + lam_y(b) + sigma(r) of this lane's columns
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const long long c = c0 + nb * 16 + l16;
    colok[nb] = c < total;
    const long long s = colok[nb] ? c / Nn : 0;
    const long long n = colok[nb] ? c - s * Nn : 0;
    base[nb] = s * K * Nn + n;
    if constexpr (EPI == EPI_DIVIDE) den_xy[nb] = colok[nb] ? column_shift(ep, n, static_cast<int>(s)) : 1.0;
  }
  f4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};
  u16x8 a_cur[MB], a_nxt[MB], b_cur[NB], b_nxt[NB];
  auto load = [&](int kb, u16x8(&a)[MB], u16x8(&b)[NB]) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      a[mb] = *reinterpret_cast<const u16x8*>(Msw + ((static_cast<long long>(rb0 + mb) * KB + kb) * 64 + lane) * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kb * 32 + 8 * g + j;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb][j] = (colok[nb] && k < K) ? X[base[nb] + static_cast<long long>(k) * Nn] : 0;
    }
  };
  load(0, a_cur, b_cur);
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + 1 < KB) load(kb + 1, a_nxt, b_nxt);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma_bf16(a_cur[mb], b_cur[nb], acc[mb][nb]);
    if (kb + 1 < KB) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a_cur[mb] = a_nxt[mb];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b_cur[nb] = b_nxt[nb];
    }
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = (rb0 + mb) * 16 + 4 * g + r;
        if (a >= K || !colok[nb]) continue;
        const long long idx = base[nb] + static_cast<long long>(a) * Nn;
        if constexpr (EPI == EPI_DIVIDE) {
          Y[idx] = store_cvt<bf16_t>(divide_by_eigs(static_cast<double>(acc[mb][nb][r]), ep, a, den_xy[nb]));
        } else {
          Y[idx] = f32_to_bf16(acc[mb][nb][r]);
        }
      }
}

// ------------------------------------------------------------------ BF16 right form
template <typename TOut, int W, int NB, int MB, int EPI, bool VEC>
__global__ __launch_bounds__(256) void k_right_bf16(const bf16_t* __restrict__ Msw, int KB, int K,
                                                    const bf16_t* __restrict__ X, TOut* __restrict__ Y,
                                                    long long Mrows, EpiArgs ep) {
  constexpr int WM = 4 / W;
  constexpr int MT = WM * MB * 16;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wn = wave % W, wm = wave / W;
  const int l16 = lane & 15, g = lane >> 4;
  const long long mwg = static_cast<long long>(blockIdx.x) * MT;
  const long long m0 = mwg + wm * MB * 16;
  const int cb0 = wn * NB;
  const bf16_t* rowp[MB];
  bool rowok[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const long long row = m0 + mb * 16 + l16;
    rowok[mb] = row < Mrows;
    rowp[mb] = X + (rowok[mb] ? row : 0) * K;
  }
  f4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};
  u16x8 a_cur[MB], a_nxt[MB], b_cur[NB], b_nxt[NB];
  auto load = [&](int kb, u16x8(&a)[MB], u16x8(&b)[NB]) {
    const int kq = kb * 32 + 8 * g;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      if constexpr (VEC) {
        a[mb] = (rowok[mb] && kq < K) ? *reinterpret_cast<const u16x8*>(rowp[mb] + kq) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[mb][j] = (rowok[mb] && kq + j < K) ? rowp[mb][kq + j] : 0;
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      b[nb] = *reinterpret_cast<const u16x8*>(Msw + ((static_cast<long long>(cb0 + nb) * KB + kb) * 64 + lane) * 8);
  };
  load(0, a_cur, b_cur);
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + 1 < KB) load(kb + 1, a_nxt, b_nxt);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mma_bf16(a_cur[mb], b_cur[nb], acc[mb][nb]);
    if (kb + 1 < KB) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a_cur[mb] = a_nxt[mb];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b_cur[nb] = b_nxt[nb];
    }
  }
  [[maybe_unused]] NormAcc na;
  [[maybe_unused]] const long long r_lo = (EPI == EPI_ACCUM) ? mwg / ep.rows_per_rhs : 0;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long m = m0 + mb * 16 + 4 * g + r;
      if (m >= Mrows) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int a = (cb0 + nb) * 16 + l16;
        if (a >= K) continue;
        const long long idx = m * K + a;
        if constexpr (EPI == EPI_ACCUM) {
          const double du = static_cast<double>(acc[mb][nb][r]);
          const double un = (ep.accum_zero ? 0.0 : static_cast<double>(Y[idx])) + du;
          Y[idx] = store_cvt<TOut>(un);
          na.add(ep, r_lo, rhs_of_row(m, r_lo, ep.rows_per_rhs), du, un);
        } else {
          Y[idx] = store_cvt<TOut>(static_cast<double>(acc[mb][nb][r]));
        }
      }
    }
  if constexpr (EPI == EPI_ACCUM) na.flush(ep, r_lo, (Mrows + ep.rows_per_rhs - 1) / ep.rows_per_rhs, lane);
}

// ------------------------------------------------------------------ launch helpers
template <typename F>
inline hipError_t for_cfg(int ci, F&& f) {
  switch (ci) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 9: return f(std::integral_constant<int, 9>{});
    default: return hipErrorInvalidValue;
  }
}

inline dim3 grid1d(long long blocks) { return dim3(static_cast<unsigned>(blocks)); }

}  // namespace helm
