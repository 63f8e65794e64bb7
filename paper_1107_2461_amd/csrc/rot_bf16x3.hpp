// Split-BF16 mode products with rotating layout (device templates).
//
// Every transform of eq. 29 is run as one GEMM form: the input is X[r][pq][k] (the
// contracted axis k contiguous, pq a flattened pair of the other two axes, r the RHS) and
// the output is Y[r][a][pq] = sum_k M[a][k] X[r][pq][k]: the contracted axis moves to the
// front.  Three such rotations restore the natural order, so the six transforms
//   x-fwd, y-fwd, z-fwd + divide, x-inv, y-inv, z-inv (+ update)
// map [k][j][i] -> [a][k][j] -> [b][a][k] -> [c][b][a] -> [i][c][b] -> [j][i][c] -> [k][j][i],
// each reading whole rows and writing 64-byte (FP32) or 128-byte (FP64) runs.  The inverse
// transforms act on different axes and commute, so running them x, y, z keeps the rotation.
//
// Arithmetic: the operands are split into three bfloat16 pieces, v = v1 + v2 + v3 with
// |v2| <~ 2^-8 |v1| and |v3| <~ 2^-16 |v1| (the eigenvector matrix once on the host, the FP32
// data on the fly), and the six partial products with i + j <= 4 are accumulated on the
// BF16 MFMA (16x16x32, FP32 accumulation), smallest first.  The dropped products are of
// relative size 2^-24, so each product is FP32-accurate (the split-BF16 scheme of Henry,
// Tang & Heinecke, ARITH 2019) at the BF16 matrix rate.  Intermediates are FP32.
//
// Workgroup: 4 waves; W of them span the K output columns (NB 16-wide blocks each), 4/W
// span the MT rows (MB 16-row blocks each).  Per 32-wide k-block the workgroup loads its
// MT x 32 FP32 input tile once (one 32-byte load per thread), splits it with the hardware
// bfloat16 conversion and stores the three pieces in LDS in MFMA fragment order (double
// buffered); every wave then reads its A fragments from LDS and its B fragments (the three
// swizzled pieces of M, shared by all workgroups, L2-resident) from global memory.
#pragma once

#include "mode_common.hpp"

namespace helm {

typedef float f8v __attribute__((ext_vector_type(8)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d8v __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_bits(float x) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));  // v_cvt_pk_bf16_f32 (RNE)
}
__device__ inline float bf16_value(unsigned short h) { return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16); }

// x = hi + mid + lo in bfloat16; the differences are exact in FP32.
__device__ inline void split3(const f8v& x, u16x8& hi, u16x8& mid, u16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = x[j];
    const unsigned short h = bf16_bits(v);
    const float r1 = v - bf16_value(h);
    const unsigned short m = bf16_bits(r1);
    hi[j] = h;
    mid[j] = m;
    lo[j] = bf16_bits(r1 - bf16_value(m));
  }
}

// TIn: float for intermediates, double when the first product reads the FP64 right-hand side
// directly (rounded to FP32 on load, as a separate conversion pass would).
template <int W, int NB, int MB, int EPI, bool VEC, typename TIn = float>
__global__ __launch_bounds__(256, 2) void k_rot_bf16x3(const bf16_t* __restrict__ Msw, long long piece, int KB, int K,
                                                       const TIn* __restrict__ X, void* __restrict__ Yv,
                                                       long long R, long long PQ, EpiArgs ep) {
  constexpr int WM = 4 / W;
  constexpr int MT = WM * MB * 16;        // rows per workgroup
  constexpr int RB = MT / 16;             // 16-row blocks per workgroup
  constexpr int CHUNKS = RB * 64;         // 8-element chunks per k-block tile
  constexpr int CPT = (CHUNKS + 255) / 256;
  __shared__ u16x8 lds[2][3][RB * 64];    // [buffer][piece][row block * 64 + lane]
  // divide: lambda_x + lambda_y + sigma of every tile row and lambda_z of every output column,
  // in FP64, staged before the main loop, so the epilogue waits on no global load
  constexpr int NSH = EPI == EPI_DIVIDE ? MT : 4;
  constexpr int NLZ = EPI == EPI_DIVIDE ? W * NB * 16 : 4;
  __shared__ __align__(16) double sh_shift[NSH];
  __shared__ double sh_lamz[NLZ];

  const int tid = threadIdx.x;
  // the wave index is uniform: keep it (and every B-fragment base address) in scalar registers
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wn = wave % W, wm = wave / W;
  const int l16 = lane & 15, g = lane >> 4;
  const long long Mrows = R * PQ;
  const long long mwg = static_cast<long long>(blockIdx.x) * MT;
  const int cb0 = wn * NB;
  const int rb0 = wm * MB;                // this wave's first row block inside the tile
  // grouped solve: the tile's rows lie inside one RHS (span = PQ), whose plan gives M and the
  // eigenvalues of the divide
  const long long rg = ep.msw_rhs ? mwg / ep.span : 0;
  const gptr_t<bf16_t> Mp = rhs_ptr(ep.msw_rhs, rg, Msw);

  // producer assignment: chunk c -> row block c / 64, fragment lane c % 64
  const TIn* src[CPT];
  bool srcok[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int c = tid + q * 256;
    const int rb = c >> 6, ln = c & 63;
    const long long row = mwg + rb * 16 + (ln & 15);
    srcok[q] = c < CHUNKS && row < Mrows;
    src[q] = X + (srcok[q] ? row : 0) * K + 8 * (ln >> 4);
  }
  // tiles are staged raw (FP32, or FP64 for the first product of a solve) and rounded to
  // FP32 when split, so a wait for a staged load never precedes the MFMA work it overlaps
  using raw_t = typename std::conditional<sizeof(TIn) == 8, d8v, f8v>::type;
  auto load_tile = [&](int kb, raw_t (&v)[CPT]) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int kq = kb * 32 + 8 * (((tid + q * 256) & 63) >> 4);
      if constexpr (VEC) {
        if (srcok[q] && kq < K) {
          v[q] = *reinterpret_cast<const raw_t*>(src[q] + kb * 32);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) v[q][j] = 0;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[q][j] = (srcok[q] && kq + j < K) ? src[q][kb * 32 + j] : TIn(0);
      }
    }
  };
  auto store_tile = [&](int buf, const raw_t (&v)[CPT]) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = tid + q * 256;
      if (c < CHUNKS) {
        f8v x;
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = static_cast<float>(v[q][j]);
        u16x8 h, m, l;
        split3(x, h, m, l);
        lds[buf][0][c] = h;
        lds[buf][1][c] = m;
        lds[buf][2][c] = l;
      }
    }
  };

  f4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};

  // B fragments (the three pieces of M) of one k-block for this wave's NB column blocks:
  // wave-uniform base + 32-bit lane offset (scalar-base addressing, one VGPR)
  const unsigned lane_off = static_cast<unsigned>(lane) * 8u;
  auto load_b = [&](int kb, u16x8 (&b)[NB][3]) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const gptr_t<bf16_t> base = Mp + (static_cast<long long>(cb0 + nb) * KB + kb) * 512;
      b[nb][0] = gload<u16x8>(base + lane_off);
      b[nb][1] = gload<u16x8>(base + piece + lane_off);
      b[nb][2] = gload<u16x8>(base + 2 * piece + lane_off);
    }
  };
  // input tiles kb+1 .. kb+DEPTH are in flight in registers while k-block kb is multiplied,
  // so the HBM latency is covered by DEPTH k-blocks of MFMA work
  constexpr int DEPTH = sizeof(TIn) == 8 ? 1 : 2;  // FP64 staging: twice the registers per tile
  raw_t stage[DEPTH][CPT];
  u16x8 bcur[NB][3];
  load_tile(0, stage[0]);
  if constexpr (EPI == EPI_DIVIDE) {
    const long long r0 = mwg / PQ;
    for (int i = tid; i < MT; i += 256) {
      const long long row = mwg + i;
      double sv = 1.0;  // rows past the end: never stored
      if (row < Mrows) {
        const long long rr = rhs_of_row(row, r0, PQ);
        sv = rhs_ptr(ep.lamxy_rhs, rr, ep.lamxy)[row - rr * PQ] + ep.sigma[rr];
      }
      sh_shift[i] = sv;
    }
    const gptr_t<double> lamz = rhs_ptr(ep.lamz_rhs, rg, ep.lamz);
    for (int a = tid; a < NLZ; a += 256) sh_lamz[a] = a < K ? lamz[a] : 1.0;
  }
  store_tile(0, stage[0]);
#pragma unroll
  for (int d = 0; d < DEPTH; ++d)
    if (1 + d < KB) load_tile(1 + d, stage[d]);
  __syncthreads();
  for (int kb = 0; kb < KB; ++kb) {
    const int buf = kb & 1;
    // B fragments of all NB column blocks stay in registers; the row blocks' A fragments are
    // read from LDS one block at a time, so a wave can cover many rows per L2 read of M
    load_b(kb, bcur);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int c = (rb0 + mb) * 64 + lane;
      const u16x8 a1 = lds[buf][0][c], a2 = lds[buf][1][c], a3 = lds[buf][2][c];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        f4 v = acc[mb][nb];
        v = mma_bf16(a3, bcur[nb][0], v);
        v = mma_bf16(a2, bcur[nb][1], v);
        v = mma_bf16(a1, bcur[nb][2], v);
        v = mma_bf16(a2, bcur[nb][0], v);
        v = mma_bf16(a1, bcur[nb][1], v);
        v = mma_bf16(a1, bcur[nb][0], v);
        acc[mb][nb] = v;
      }
    }
    if (kb + 1 < KB) {
      store_tile(buf ^ 1, stage[0]);
#pragma unroll
      for (int d = 0; d + 1 < DEPTH; ++d)
#pragma unroll
        for (int q = 0; q < CPT; ++q) stage[d][q] = stage[d + 1][q];
      if (kb + 1 + DEPTH < KB) load_tile(kb + 1 + DEPTH, stage[DEPTH - 1]);
    }
    __syncthreads();
  }

  // epilogue: lane holds rows m = mwg + (rb0 + mb)*16 + 4g + t (t < 4), column a = (cb0 + nb)*16 + l16
  const long long r_lo = mwg / PQ;
  [[maybe_unused]] double lamz_c[EPI == EPI_DIVIDE ? NB : 1];
  if constexpr (EPI == EPI_DIVIDE) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) lamz_c[nb] = sh_lamz[(cb0 + nb) * 16 + l16];
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const long long mq = mwg + (rb0 + mb) * 16 + 4 * g;  // first of the lane's four rows
    [[maybe_unused]] double shift[4];
    if constexpr (EPI == EPI_DIVIDE) {
#pragma unroll
      for (int t = 0; t < 4; ++t) shift[t] = sh_shift[(rb0 + mb) * 16 + 4 * g + t];
    }
    long long rr[4], pq[4];
    if (PQ >= MT) {  // at most one RHS boundary inside the tile: branch-free split
      const long long o = mq - r_lo * PQ;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool nxt = o + t >= PQ;
        rr[t] = r_lo + nxt;
        pq[t] = nxt ? o + t - PQ : o + t;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        rr[t] = rhs_of_row(mq + t, r_lo, PQ);
        pq[t] = mq + t - rr[t] * PQ;
      }
    }
    const bool full = VEC && (mq + 3 < Mrows);  // the four rows share one RHS and are aligned
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int a = (cb0 + nb) * 16 + l16;
      if (a >= K) continue;
      if constexpr (EPI == EPI_STORE_F64) {
        double* Y = static_cast<double*>(Yv);
        const f4 v = acc[mb][nb];
        if (full) {
          *reinterpret_cast<d4v*>(Y + (rr[0] * K + a) * PQ + pq[0]) =
              d4v{static_cast<double>(v[0]), static_cast<double>(v[1]), static_cast<double>(v[2]),
                  static_cast<double>(v[3])};
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (mq + t < Mrows) Y[(rr[t] * K + a) * PQ + pq[t]] = static_cast<double>(v[t]);
        }
      } else {
        float* Y = static_cast<float*>(Yv);
        f4 v = acc[mb][nb];
        if constexpr (EPI == EPI_DIVIDE) {
          // eqs. 26-28: the denominator summed in FP64 and rounded once to FP32 (an exact FP64
          // zero, the Neumann null mode, is tested before rounding), then the FP32 hardware
          // reciprocal (1 ulp): at the precision of the FP32 data it divides
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double d = lamz_c[nb] + shift[t];
            v[t] = d == 0.0 ? (ep.eq28 ? v[t] : 0.f) : v[t] * __builtin_amdgcn_rcpf(static_cast<float>(d));
          }
        }
        if (full) {
          *reinterpret_cast<f4*>(Y + (rr[0] * K + a) * PQ + pq[0]) = v;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (mq + t < Mrows) Y[(rr[t] * K + a) * PQ + pq[t]] = v[t];
        }
      }
    }
  }
}

// Row blocks per wave for the rotating kernel with table entry c: 128-row workgroup tiles
// (64 for the widest entry), so the double-buffered split tile (6 bytes per element) takes at
// most 48 KB of LDS and each L2 read of M serves 128 rows.
constexpr int rot_rows(Cfg c) { return c.W == 4 ? (c.MB >= 8 ? 2 : 8) : (c.W == 2 ? 4 : 2); }

}  // namespace helm
