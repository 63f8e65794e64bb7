// gfx950 kernels of the fast-diagonalization solve path other than the mode-product
// templates (mode_common.hpp): precision dispatch of the mode products, the batched Thomas
// solve of the TPT variant, the FP64 7-point operator/residual and small helpers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "mode_common.hpp"

namespace helm {

hipError_t mode_left_f64(int, const void*, int, const void*, void*, long long, long long, Epi, const EpiArgs&,
                         hipStream_t);
hipError_t mode_left_f32(int, const void*, int, const void*, void*, long long, long long, Epi, const EpiArgs&,
                         hipStream_t);
hipError_t mode_left_bf16(int, const void*, int, const void*, void*, long long, long long, Epi, const EpiArgs&,
                          hipStream_t);
hipError_t mode_right_f64(int, const void*, int, const void*, void*, long long, Epi, bool, const EpiArgs&, hipStream_t);
hipError_t mode_right_f32(int, const void*, int, const void*, void*, long long, Epi, bool, const EpiArgs&, hipStream_t);
hipError_t mode_right_bf16(int, const void*, int, const void*, void*, long long, Epi, bool, const EpiArgs&,
                           hipStream_t);

static size_t elem_bytes(Prec p) { return p == P_F64 ? 8 : (p == P_F32 ? 4 : 2); }
static int padded_rows(int K) {
  const int c = choose_cfg(K);
  return c < 0 ? -1 : cfg_extent(kCfgs[c]);
}

size_t swizzled_bytes(Prec p, int K) {
  const int R = padded_rows(K);
  if (R < 0) return 0;
  const int kb = kblock(p);
  const int KP = (K + kb - 1) / kb * kb;
  return static_cast<size_t>(R) * KP * elem_bytes(p);
}

void swizzle_operand(Prec p, int K, const double* M, void* out) {
  const int R = padded_rows(K);
  const int kbw = kblock(p);
  const int KB = (K + kbw - 1) / kbw;
  const int per = p == P_BF16 ? 8 : 4;  // values per lane per fragment
  for (int rb = 0; rb < R / 16; ++rb)
    for (int kb = 0; kb < KB; ++kb)
      for (int lane = 0; lane < 64; ++lane)
        for (int s = 0; s < per; ++s) {
          const int row = rb * 16 + (lane & 15);
          const int k = kb * kbw + per * (lane >> 4) + s;
          const double v = (row < K && k < K) ? M[static_cast<size_t>(row) * K + k] : 0.0;
          const size_t o = ((static_cast<size_t>(rb) * KB + kb) * 64 + lane) * per + s;
          if (p == P_F64)
            static_cast<double*>(out)[o] = v;
          else if (p == P_F32)
            static_cast<float*>(out)[o] = static_cast<float>(v);
          else
            static_cast<bf16_t*>(out)[o] = f32_to_bf16(static_cast<float>(v));
        }
}

hipError_t mode_rot_bf16x3(int, const void*, long long, int, const void*, bool, void*, long long, long long, Epi,
                           bool, const EpiArgs&, hipStream_t);

size_t swizzled_bf16x3_bytes(int K) { return 3 * swizzled_bytes(P_BF16, K); }

void swizzle_bf16x3(int K, const double* M, void* out) {
  // M = M1 + M2 + M3, each piece the bfloat16 rounding of what the previous ones leave
  const size_t n = static_cast<size_t>(K) * K;
  std::vector<double> rem(M, M + n), piece(n);
  const size_t stride = swizzled_bytes(P_BF16, K);
  for (int p = 0; p < 3; ++p) {
    for (size_t i = 0; i < n; ++i) {
      piece[i] = static_cast<double>(bf16_to_f32(f32_to_bf16(static_cast<float>(rem[i]))));
      rem[i] -= piece[i];
    }
    swizzle_operand(P_BF16, K, piece.data(), static_cast<unsigned char*>(out) + p * stride);
  }
}

hipError_t mode_rot(const void* Msw, int K, const void* X, bool x_f64, void* Y, long long R, long long PQ, Epi epi,
                    const EpiArgs& ep, hipStream_t st) {
  const int ci = choose_cfg(K);
  if (ci < 0 || K < 1 || R < 1 || PQ < 1 || R > kMaxRhs) return hipErrorInvalidValue;
  if ((R * PQ + 15) / 16 > 0x7fffffffLL) return hipErrorInvalidValue;
  if (epi == EPI_ACCUM) return hipErrorInvalidValue;  // refinement updates use update_u
  const bool vec = (K % 8 == 0) && (PQ % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 64 == 0) &&
                   (reinterpret_cast<uintptr_t>(Y) % 32 == 0);
  const long long piece = static_cast<long long>(swizzled_bytes(P_BF16, K) / 2);
  return mode_rot_bf16x3(ci, Msw, piece, K, X, x_f64, Y, R, PQ, epi, vec, ep, st);
}

hipError_t mode_left(Prec p, const void* Msw, int K, const void* X, Prec tin, void* Y, Prec tout, long long S,
                     long long Nn, Epi epi, const EpiArgs& ep, hipStream_t st) {
  const int ci = choose_cfg(K);
  if (ci < 0 || K < 1 || S < 0 || Nn < 0 || tin != p || tout != p) return hipErrorInvalidValue;
  if (epi != EPI_STORE && epi != EPI_DIVIDE) return hipErrorInvalidValue;
  if ((S * Nn + 15) / 16 > 0x7fffffffLL) return hipErrorInvalidValue;
  if (p == P_F64) return mode_left_f64(ci, Msw, K, X, Y, S, Nn, epi, ep, st);
  if (ep.msw_rhs) return hipErrorInvalidValue;  // grouped solves: FP64 and split-BF16 only
  if (p == P_F32) return mode_left_f32(ci, Msw, K, X, Y, S, Nn, epi, ep, st);
  return mode_left_bf16(ci, Msw, K, X, Y, S, Nn, epi, ep, st);
}

hipError_t mode_right(Prec p, const void* Msw, int K, const void* X, Prec tin, void* Y, Prec tout, long long Mrows,
                      Epi epi, const EpiArgs& ep, hipStream_t st) {
  const int ci = choose_cfg(K);
  if (ci < 0 || K < 1 || Mrows < 0 || tin != p) return hipErrorInvalidValue;
  if ((Mrows + 15) / 16 > 0x7fffffffLL) return hipErrorInvalidValue;
  if (epi == EPI_STORE) {
    if (tout != p) return hipErrorInvalidValue;
  } else if (epi == EPI_ACCUM) {
    if (p == P_F64 || tout != P_F64 || ep.norms == nullptr || ep.rows_per_rhs < 1) return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  const int vw = p == P_BF16 ? 8 : 4;  // elements per vector load of one row
  const bool vec = (K % vw == 0) && (reinterpret_cast<uintptr_t>(X) % (vw * elem_bytes(p)) == 0);
  if (p == P_F64) return mode_right_f64(ci, Msw, K, X, Y, Mrows, epi, vec, ep, st);
  if (ep.msw_rhs) return hipErrorInvalidValue;  // grouped solves: FP64 and split-BF16 only
  if (p == P_F32) return mode_right_f32(ci, Msw, K, X, Y, Mrows, epi, vec, ep, st);
  return mode_right_bf16(ci, Msw, K, X, Y, Mrows, epi, vec, ep, st);
}

// ------------------------------------------------------------------ Thomas along z
// Two lanes per (r, b, a) line, in a two-sided (twisted) factorisation: lanes 0-31 of a wave
// eliminate 32 consecutive lines downward from the first plane, lanes 32-63 eliminate the same
// lines upward from the last plane.  Each half stops next to the middle row m = nz / 2, the
// halves trade their last inverse pivot and right-hand side with one cross-half shuffle, both
// solve row m, and each back-substitutes outward.  This halves the dependent chain of a line
// and doubles the lanes working on it; at each step a half-wave touches 32 consecutive lines of
// one z-plane (256 B).  Forward elimination keeps only a checkpoint of (1 / pivot, rhs) every
// kSeg steps; the backward sweep recomputes one segment at a time into registers, so a line is
// read twice and written once (24 B/point), in place.  The kSeg values of a segment are loaded
// together and the next segment's loads are issued before the current one is eliminated.
// Pivots are inverted once (hardware reciprocal + two Newton steps, a few ulp; the systems are
// diagonally dominant) and both sweeps multiply by the inverse.  The z operator's rows are
// staged in LDS once per workgroup.
constexpr int kSeg = 16;

namespace {
long long thomas_lanes(long long nl) { return (nl + 31) / 32 * 64; }
int thomas_nseg(int nz) { return (nz / 2 + kSeg - 1) / kSeg; }
}  // namespace

// Lines of up to kPartMaxN rows, when there are too few of them for two waves per SIMD in the
// two-sided kernel (fewer than kPartMaxLines lines), use the partitioned kernel below (segments
// of kPartSeg rows, no checkpoints); otherwise the checkpointed two-sided kernel.  Measured:
// 128^3 x 3 (49152 lines of 128) 32.0 against 34-37 us; a 256^3 cylinder (65536 radial lines of
// 256) 81.6 against 77 us, where the two-sided kernel already fills the chip.
constexpr int kPartSeg = 16;
constexpr int kPartMaxP = 16;
constexpr int kPartMaxN = kPartSeg * kPartMaxP;
constexpr long long kPartMaxLines = 65536;

namespace {
bool thomas_partitioned(int nz, long long nl) { return nz <= kPartMaxN && nl < kPartMaxLines; }
}  // namespace

size_t thomas_scratch_bytes(int nx, int ny, int nz, int nrhs) {
  const long long nl = static_cast<long long>(nx) * ny * nrhs;
  if (thomas_partitioned(nz, nl)) return 0;
  return static_cast<size_t>(2LL * thomas_nseg(nz) * thomas_lanes(nl)) * sizeof(double);
}

// CYL: the cylindrical line operator K_r + lam_theta G + (lam_z + sigma) V_r (eq. 44).
template <bool CYL>
__global__ __launch_bounds__(64) void k_thomas(double* __restrict__ v, ThomasArgs a, double* __restrict__ chk) {
  // K_z diagonal [nz], V_z [nz], K_z off-diagonal [nz] (last = 0), and for CYL the metric G [nz]
  extern __shared__ double zrow[];
  const int nz = a.nz;
  double* sk = zrow;
  double* sv = zrow + nz;
  double* so = zrow + 2 * nz;
  double* sg = zrow + 3 * nz;
  for (int i = threadIdx.x; i < nz; i += 64) {
    sk[i] = a.kdiag[i];
    sv[i] = a.vol[i];
    so[i] = i < nz - 1 ? a.koff[i] : 0.0;
    if constexpr (CYL) sg[i] = a.gdiag[i];
  }
  __syncthreads();
  const long long Nn = static_cast<long long>(a.nx) * a.ny;
  const long long nl = Nn * a.nrhs;
  const int bot = threadIdx.x >> 5;  // 0: from the first plane down; 1: from the last plane up
  const long long line = static_cast<long long>(blockIdx.x) * 32 + (threadIdx.x & 31);
  const long long lane_id = static_cast<long long>(blockIdx.x) * 64 + threadIdx.x;
  const long long nlanes = static_cast<long long>(gridDim.x) * 64;
  // both lanes of a line leave together, so the middle-row shuffle only reads live partners
  if (line >= nl) return;
  const int r = static_cast<int>(line / Nn);
  const long long n = line - r * Nn;
  if (a.skip_null && n == 0) return;
  const int ax = static_cast<int>(n % a.nx), by = static_cast<int>(n / a.nx);
  // diagonal of row k: K_kk + c V_k (+ cg G_k for CYL)
  const double c = CYL ? a.lamy[by] + a.sigma[r] : a.lamx[ax] + a.lamy[by] + a.sigma[r];
  const double cg = CYL ? a.lamx[ax] : 0.0;
  const int m = nz / 2;
  const int len = bot ? nz - 1 - m : m;  // rows this lane eliminates: m above the middle, the rest below
  const long long stride = bot ? -Nn : Nn;
  double* col0 = v + static_cast<long long>(r) * nz * Nn + n;
  double* base = bot ? col0 + static_cast<long long>(nz - 1) * Nn : col0;
  const int nseg = (m + kSeg - 1) / kSeg;
  // row of step s, and the LDS index of the off-diagonal entry joining steps s - 1 and s
  auto row_of = [&](int s) { return min(max(bot ? nz - 1 - s : s, 0), nz - 1); };
  auto cpl_of = [&](int s) { return min(max(bot ? nz - 1 - s : s - 1, 0), nz - 1); };
  auto load_seg = [&](int j, double (&g)[kSeg]) {
#pragma unroll
    for (int t = 0; t < kSeg; ++t) {
      const int s = j * kSeg + t;
      g[t] = s < len ? base[s * stride] : 0.0;
    }
  };
  // elimination of one segment from the carried (1 / beta, y): fills ib[t] = 1 / beta_s and
  // ys[t] = y_s, with beta_s = D_s - Koff_s^2 / beta_{s-1}, y_s = V_s g_s - m_s y_{s-1}.  The
  // segment's operator entries are read and its diagonals and right-hand sides formed before
  // the recurrence, so no load sits inside the dependent chain.
  auto eliminate = [&](int j, const double (&g)[kSeg], double& ibeta, double& y, double (&ib)[kSeg],
                       double (&ys)[kSeg]) {
    double dg[kSeg], rh[kSeg], ko[kSeg];
#pragma unroll
    for (int t = 0; t < kSeg; ++t) {
      const int s = j * kSeg + t;
      const int rw = row_of(s);
      const double vk = sv[rw];
      dg[t] = CYL ? sk[rw] + c * vk + cg * sg[rw] : sk[rw] + c * vk;
      rh[t] = vk * g[t];
      ko[t] = so[cpl_of(s)];
    }
#pragma unroll
    for (int t = 0; t < kSeg; ++t) {
      const int s = j * kSeg + t;
      if (s < len) {
        if (s == 0) {
          ibeta = recip(dg[t]);
          y = rh[t];
        } else {
          const double mu = ko[t] * ibeta;
          ibeta = recip(dg[t] - mu * ko[t]);
          y = rh[t] - mu * y;
        }
      }
      ib[t] = ibeta;
      ys[t] = y;
    }
  };
  double g0[kSeg], g1[kSeg], ib[kSeg], ys[kSeg];
  double ibeta = 0.0, y = 0.0;  // stays 0 on a side with no rows
  // forward sweep, checkpoints at the end of every segment but the last; the loop is unrolled
  // by two so the two segment buffers swap roles without a copy (a copy would wait for the
  // prefetch just issued)
  auto fwd = [&](int j, const double (&cur)[kSeg], double (&nxt)[kSeg]) {
    if (j + 1 < nseg) load_seg(j + 1, nxt);
    eliminate(j, cur, ibeta, y, ib, ys);
    if (j + 1 < nseg) {
      chk[(2LL * j) * nlanes + lane_id] = ibeta;
      chk[(2LL * j + 1) * nlanes + lane_id] = y;
    }
  };
  if (nseg > 0) load_seg(0, g0);
  for (int j = 0; j < nseg; j += 2) {
    fwd(j, g0, g1);
    if (j + 1 < nseg) fwd(j + 1, g1, g0);
  }
  // the middle row, from both eliminated sides (computed in the same order by both lanes)
  const double ib_p = __shfl_xor(ibeta, 32), y_p = __shfl_xor(y, 32);
  const double ib_t = bot ? ib_p : ibeta, y_t = bot ? y_p : y;
  const double ib_b = bot ? ibeta : ib_p, y_b = bot ? y : y_p;
  const double o_t = so[max(m - 1, 0)], o_b = so[m];  // couplings of row m to rows m - 1 and m + 1
  const double mt = o_t * ib_t, mb = o_b * ib_b;
  const double vm = sv[m];
  const double dm = (CYL ? sk[m] + c * vm + cg * sg[m] : sk[m] + c * vm) - mt * o_t - mb * o_b;
  const double xm = (vm * col0[static_cast<long long>(m) * Nn] - mt * y_t - mb * y_b) / dm;
  if (!bot) col0[static_cast<long long>(m) * Nn] = xm;
  // backward sweep, one segment at a time from the middle outward.  The checkpoint a segment
  // starts from is loaded one segment ahead, before that segment's values: loads retire in
  // issue order, so the state is in registers when its segment is eliminated.
  double xnext = xm;
  double ib_in = 0.0, y_in = 0.0;  // state entering the segment being eliminated
  auto load_chk = [&](int j, double& ibc, double& yc) {  // state entering segment j (j > 0)
    ibc = chk[(2LL * (j - 1)) * nlanes + lane_id];
    yc = chk[(2LL * (j - 1) + 1) * nlanes + lane_id];
  };
  auto bwd = [&](int j, const double (&cur)[kSeg], double (&nxt)[kSeg]) {
    double ib_nx = 0.0, y_nx = 0.0;
    if (j > 1) load_chk(j - 1, ib_nx, y_nx);
    if (j > 0) load_seg(j - 1, nxt);
    ibeta = ib_in;
    y = y_in;
    eliminate(j, cur, ibeta, y, ib, ys);
    double kup[kSeg];  // off-diagonal joining step s with step s + 1 (the middle row after the last)
#pragma unroll
    for (int t = 0; t < kSeg; ++t) kup[t] = so[cpl_of(j * kSeg + t + 1)];
#pragma unroll
    for (int t = kSeg - 1; t >= 0; --t) {
      const int s = j * kSeg + t;
      if (s < len) {
        const double xs = (ys[t] - kup[t] * xnext) * ib[t];
        base[s * stride] = xs;
        xnext = xs;
      }
    }
    ib_in = ib_nx;
    y_in = y_nx;
  };
  if (nseg > 1) load_chk(nseg - 1, ib_in, y_in);
  if (nseg > 0) load_seg(nseg - 1, g0);
  for (int j = nseg - 1; j >= 0; j -= 2) {
    bwd(j, g0, g1);
    if (j - 1 >= 0) bwd(j - 1, g1, g0);
  }
}

// Partitioned line solve for lines of up to kPartMaxN rows: each line is cut into P segments of
// kPartSeg rows, one lane per segment, and a workgroup holds 64 lines x P segments (wave w =
// segment w of 64 consecutive lines, so every row access of a wave is 64 consecutive values of
// one plane).  This gives P times the lanes of one chain per line and chains of kPartSeg steps:
//   1. each segment expresses its first and last unknowns through the unknowns just outside it,
//      x_first = YF + ZF xL + WF xR and x_last = YL + ZL xL + WL xR, by one elimination from the
//      top (its pivots kept) and one from the bottom;
//   2. one lane per line solves the 2P interface equations by a two-term recurrence over the
//      segments and back-substitution (the reduced system of a diagonally dominant line is
//      diagonally dominant, so no pivoting);
//   3. each segment solves its rows with xL and xR known (the top pivots reused).
// Each value is read once and written once (16 B per point), in place.

template <bool CYL>
__global__ __launch_bounds__(64 * kPartMaxP) void k_thomas_part(double* __restrict__ v, ThomasArgs a, int P) {
  extern __shared__ double shm[];
  const int nz = a.nz;
  double* sk = shm;                 // K diagonal [nz]
  double* sv = shm + nz;            // V [nz]
  double* so = shm + 2 * nz;        // K off-diagonal [nz] (last = 0)
  double* sg = shm + 3 * nz;        // CYL: the metric G [nz]
  // [P][6][64] per segment and line: YF ZF WF YL ZL WL, then (step 2) d e al ga and finally
  // x_first x_last in slots 4 and 5
  double* red = shm + 4 * nz;
  for (int i = threadIdx.x; i < nz; i += blockDim.x) {
    sk[i] = a.kdiag[i];
    sv[i] = a.vol[i];
    so[i] = i < nz - 1 ? a.koff[i] : 0.0;
    if constexpr (CYL) sg[i] = a.gdiag[i];
  }
  __syncthreads();
  const long long Nn = static_cast<long long>(a.nx) * a.ny;
  const long long nl = Nn * a.nrhs;
  const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const long long line = static_cast<long long>(blockIdx.x) * 64 + lane;
  // lanes of absent or skipped lines do no memory access but take part in every barrier
  bool act = line < nl;
  const int r = act ? static_cast<int>(line / Nn) : 0;
  const long long n = act ? line - r * Nn : 0;
  if (a.skip_null && n == 0) act = false;
  const int ax = static_cast<int>(n % a.nx), by = static_cast<int>(n / a.nx);
  const double c = CYL ? a.lamy[by] + a.sigma[r] : a.lamx[ax] + a.lamy[by] + a.sigma[r];
  const double cg = CYL ? a.lamx[ax] : 0.0;
  const int lo = seg * kPartSeg;
  const int len = max(0, min(kPartSeg, nz - lo));
  double* col = v + static_cast<long long>(r) * nz * Nn + n;
  auto diag = [&](int i) { return CYL ? sk[i] + c * sv[i] + cg * sg[i] : sk[i] + c * sv[i]; };
  // the segment's right-hand side V g, all loads issued before the recurrences
  double rh[kPartSeg];
#pragma unroll
  for (int t = 0; t < kPartSeg; ++t) rh[t] = (act && t < len) ? col[static_cast<long long>(lo + t) * Nn] : 0.0;
#pragma unroll
  for (int t = 0; t < kPartSeg; ++t) rh[t] *= (t < len) ? sv[lo + t] : 0.0;
  const double cl = lo > 0 ? so[lo - 1] : 0.0;               // coupling to x_{lo - 1}
  const double cr = len > 0 ? so[lo + len - 1] : 0.0;        // coupling to x_{lo + len} (0 at the end)
  // 1a. elimination from the top: pivots (kept), the right-hand side and the left spike
  double ib[kPartSeg];
  double y = 0.0, z = 0.0, ibp = 0.0;
#pragma unroll
  for (int t = 0; t < kPartSeg; ++t) {
    if (t < len) {
      const int i = lo + t;
      if (t == 0) {
        ibp = recip(diag(i));
        y = rh[0];
        z = -cl;
      } else {
        const double mu = so[i - 1] * ibp;
        ibp = recip(diag(i) - mu * so[i - 1]);
        y = rh[t] - mu * y;
        z = -mu * z;
      }
    }
    ib[t] = ibp;
  }
  const double YL = y * ibp, ZL = z * ibp, WL = -cr * ibp;
  // 1b. elimination from the bottom: the right-hand side and the right spike
  double yb = 0.0, w = 0.0, ibb = 0.0;
#pragma unroll
  for (int t = kPartSeg - 1; t >= 0; --t) {
    if (t < len) {
      const int i = lo + t;
      if (t == len - 1) {
        ibb = recip(diag(i));
        yb = rh[t];
        w = -cr;
      } else {
        const double mu = so[i] * ibb;
        ibb = recip(diag(i) - mu * so[i]);
        yb = rh[t] - mu * yb;
        w = -mu * w;
      }
    }
  }
  const double YF = yb * ibb, WF = w * ibb, ZF = -cl * ibb;
  double* rs = red + (6 * seg) * 64 + lane;
  rs[0] = YF;
  rs[64] = ZF;
  rs[128] = WF;
  rs[192] = YL;
  rs[256] = ZL;
  rs[320] = WL;
  __syncthreads();
  // 2. interface unknowns of the line (wave 0): with L_{s-1} = d + e F_s carried,
  //    F_s = al_s + ga_s F_{s+1}, L_s = d_s + e_s F_{s+1}
  if (seg == 0) {
    double d = 0.0, e = 0.0;
    for (int s2 = 0; s2 < P; ++s2) {
      const double* q = red + (6 * s2) * 64 + lane;
      const double yf = q[0], zf = q[64], wf = q[128], yl = q[192], zl = q[256], wl = q[320];
      const double den = 1.0 / (1.0 - zf * e);
      const double al = (yf + zf * d) * den, ga = wf * den;
      const double dn = yl + zl * (d + e * al), en = zl * e * ga + wl;
      // keep (d, e, al, ga) of segment s2 (its slots are read) for the back-substitution
      double* o = red + (6 * s2) * 64 + lane;
      o[0] = dn;
      o[64] = en;
      o[128] = al;
      o[192] = ga;
      d = dn;
      e = en;
    }
    double F = 0.0;  // F_P: no segment beyond the last
    for (int s2 = P - 1; s2 >= 0; --s2) {
      double* o = red + (6 * s2) * 64 + lane;
      const double L = o[0] + o[64] * F;  // L_s with F_{s+1}
      F = o[128] + o[192] * F;            // F_s
      o[256] = F;
      o[320] = L;
    }
  }
  __syncthreads();
  // 3. the segment with its outside neighbours known: x_{lo-1} = L_{seg-1}, x_{lo+len} = F_{seg+1}
  const double xL = seg > 0 ? red[(6 * (seg - 1) + 5) * 64 + lane] : 0.0;
  const double xR = seg + 1 < P ? red[(6 * (seg + 1) + 4) * 64 + lane] : 0.0;
  double ys[kPartSeg];
  double yy = 0.0;
#pragma unroll
  for (int t = 0; t < kPartSeg; ++t) {
    if (t < len) {
      double rt = rh[t];
      if (t == 0) rt -= cl * xL;
      if (t == len - 1) rt -= cr * xR;
      yy = t == 0 ? rt : rt - so[lo + t - 1] * ib[t - 1] * yy;
    }
    ys[t] = yy;
  }
  double xn = 0.0;
#pragma unroll
  for (int t = kPartSeg - 1; t >= 0; --t) {
    if (t < len) {
      const double xt = (t == len - 1) ? ys[t] * ib[t] : (ys[t] - so[lo + t] * xn) * ib[t];
      if (act) col[static_cast<long long>(lo + t) * Nn] = xt;
      xn = xt;
    }
  }
}

hipError_t thomas_z(double* v, const ThomasArgs& a, void* chk, hipStream_t st) {
  const long long nl = static_cast<long long>(a.nx) * a.ny * a.nrhs;
  if (nl == 0) return hipSuccess;
  if (a.nz < 1 || a.nz > 2048) return hipErrorInvalidValue;
  if (thomas_partitioned(a.nz, nl)) {  // partitioned lines: P segments of kPartSeg rows
    const int P = (a.nz + kPartSeg - 1) / kPartSeg;
    const long long blocks = (nl + 63) / 64;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = (4 * static_cast<size_t>(a.nz) + 6 * 64 * static_cast<size_t>(P)) * sizeof(double);
    if (a.gdiag)
      hipLaunchKernelGGL(k_thomas_part<true>, dim3(static_cast<unsigned>(blocks)), dim3(64 * P), lds, st, v, a, P);
    else
      hipLaunchKernelGGL(k_thomas_part<false>, dim3(static_cast<unsigned>(blocks)), dim3(64 * P), lds, st, v, a, P);
    return hipGetLastError();
  }
  const long long blocks = thomas_lanes(nl) / 64;
  const size_t lds = (a.gdiag ? 4 : 3) * static_cast<size_t>(a.nz) * sizeof(double);
  if (a.gdiag)
    hipLaunchKernelGGL(k_thomas<true>, dim3(static_cast<unsigned>(blocks)), dim3(64), lds, st, v, a,
                       static_cast<double*>(chk));
  else
    hipLaunchKernelGGL(k_thomas<false>, dim3(static_cast<unsigned>(blocks)), dim3(64), lds, st, v, a,
                       static_cast<double*>(chk));
  return hipGetLastError();
}

// ------------------------------------------------------------------ singular z line (TPT, all-Neumann)
// The (0, 0) line of every RHS through its eigenbasis: ghat = E^{-1} g, the divide (the zero
// eigenvalue projected, or eq. 28), u = E ghat.  Two launches spread the two matrix-vector
// products over many workgroups: one wave per matrix row, its lanes reading the row at
// consecutive addresses, a fixed shuffle tree summing them.
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ghat[r][c] = (E^{-1} g)_c / lambda_c (0 or the sum itself for lambda_c = 0), c = 4 blockIdx.x + wave
__global__ __launch_bounds__(256) void k_null_fwd(const double* __restrict__ v, const double* __restrict__ Ezinv,
                                                  const double* __restrict__ lamz, double* __restrict__ gh, int nx,
                                                  int ny, int nz, int eq28) {
  const int r = blockIdx.y;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= nz) return;  // whole waves leave together
  const long long Nn = static_cast<long long>(nx) * ny;
  const double* col = v + static_cast<long long>(r) * nz * Nn;  // line (a, b) = (0, 0)
  double s = 0.0;
  for (int k = lane; k < nz; k += 64) s += Ezinv[static_cast<long long>(c) * nz + k] * col[static_cast<long long>(k) * Nn];
  s = wave_sum(s);
  if (lane == 0) {
    const double lam = lamz[c];  // the shift of this line is lam_x(0) + lam_y(0) + sigma = 0
    gh[static_cast<long long>(r) * nz + c] = (lam == 0.0) ? (eq28 ? s : 0.0) : s / lam;
  }
}

// u[r][k] = (E ghat)_k on the line, k = 4 blockIdx.x + wave
__global__ __launch_bounds__(256) void k_null_inv(double* __restrict__ v, const double* __restrict__ Ez,
                                                  const double* __restrict__ gh, int nx, int ny, int nz) {
  const int r = blockIdx.y;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (k >= nz) return;
  const long long Nn = static_cast<long long>(nx) * ny;
  const double* g = gh + static_cast<long long>(r) * nz;
  double s = 0.0;
  for (int c = lane; c < nz; c += 64) s += Ez[static_cast<long long>(k) * nz + c] * g[c];
  s = wave_sum(s);
  if (lane == 0) v[static_cast<long long>(r) * nz * Nn + static_cast<long long>(k) * Nn] = s;
}

hipError_t null_line_z(double* v, const double* Ez, const double* Ezinv, const double* lamz, int nx, int ny, int nz,
                       int nrhs, int eq28, double* scratch, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (!scratch || nrhs > 65535) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((nz + 3) / 4), static_cast<unsigned>(nrhs));
  hipLaunchKernelGGL(k_null_fwd, grid, dim3(256), 0, st, v, Ezinv, lamz, scratch, nx, ny, nz, eq28);
  hipLaunchKernelGGL(k_null_inv, grid, dim3(256), 0, st, v, Ez, scratch, nx, ny, nz);
  return hipGetLastError();
}

// ------------------------------------------------------------------ 7-point operator / residual
// Column segments: a lane owns one x index and kStencilJS consecutive y rows and marches up a
// z-chunk, keeping the rows of planes k-1, k (with the two y-halo rows) and k+1 in registers.
// The x neighbours come from the adjacent lanes (cross-lane shuffle); only the two edge lanes
// of a wave load one value each.  A workgroup is 4 waves: wx of them side by side in x (64 x
// indices each) times 4 / wx row segments.  Workgroups are numbered so that each XCD (which
// receives every 8th workgroup) walks a contiguous range of tiles, y fastest then z: the halo
// rows and planes a tile shares with its neighbours are then read while they sit in that
// XCD's L2.  Per point: 8 B of u, 8 B of f in, one value out, plus halo re-reads.  Two rows
// per lane: one reads the halo rows 3x over, four hold more registers (fewer waves per SIMD).
constexpr int kStencilJS = 2;

template <typename T>
__device__ inline T lane_below(T v, int lane) { return __shfl(v, lane > 0 ? lane - 1 : 0); }
template <typename T>
__device__ inline T lane_above(T v, int lane) { return __shfl(v, lane < 63 ? lane + 1 : 63); }

// TU: storage of u (FP64, or FP32 for the first solve's result, which is exact in FP64 once read)
// CYL: cylindrical operator (x = theta, y = z, z = r): the x term of plane k is scaled by
// a.xscale[k], and x is periodic when a.xper is set.
template <typename TOut, int MODE, typename TU, bool CYL = false>  // MODE 0: out = H u, 1: out = f - H u
__global__ __launch_bounds__(256) void k_stencil(const TU* __restrict__ u,
                                                 const double* __restrict__ f, TOut* __restrict__ out,
                                                 StencilArgs a, int zchunk, int nzc, int wx, int nbx, int nby) {
  constexpr int JS = kStencilJS;
  if (a.zero && blockIdx.x == 0)
    for (int q = threadIdx.x; q < a.nzero; q += blockDim.x) a.zero[q] = 0ull;
  // the wave index is uniform: the row segment (and its coefficients) then live in SGPRs
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nt = gridDim.x;
  const int per = nt / 8;
  int t = blockIdx.x;
  if (per > 0 && t < per * 8) t = (t % 8) * per + t / 8;
  const int bxx = t % nbx;
  t /= nbx;
  const int byy = t % nby;
  t /= nby;
  const int zc = t % nzc;
  const int r = t / nzc;
  const int i = (bxx * wx + w % wx) * 64 + lane;
  const int j0 = (byy * (4 / wx) + w / wx) * JS;
  const int k0 = zc * zchunk;
  const int k1 = min(a.nz, k0 + zchunk);
  if (k0 >= k1 || j0 >= a.ny) return;
  const bool iok = i < a.nx;
  const int ic = iok ? i : a.nx - 1;  // lanes past the end load a valid column, store nothing
  const long long plane = static_cast<long long>(a.nx) * a.ny;
  const long long rbase = static_cast<long long>(r) * plane * a.nz;
  const gptr_t<double> cx = rhs_ptr(a.cx_rhs, r, a.cx);
  const gptr_t<double> cy = rhs_ptr(a.cy_rhs, r, a.cy);
  const gptr_t<double> cz = rhs_ptr(a.cz_rhs, r, a.cz);
  const double cxl = cx[3 * ic], cxd = cx[3 * ic + 1], cxu = cx[3 * ic + 2];
  const bool xper = CYL && a.xper;
  const bool hx_lo = xper || ic > 0, hx_hi = xper || ic + 1 < a.nx;
  int jr[JS + 2];  // rows j0-1 .. j0+JS, clamped into the grid
#pragma unroll
  for (int s = 0; s < JS + 2; ++s) jr[s] = min(max(j0 - 1 + s, 0), a.ny - 1);
  double cyl[JS], cyu[JS], dxy[JS];
#pragma unroll
  for (int s = 0; s < JS; ++s) {
    const int j = jr[s + 1];
    cyl[s] = (j0 + s > 0 && j0 + s < a.ny) ? cy[3 * j] : 0.0;
    cyu[s] = (j0 + s + 1 < a.ny) ? cy[3 * j + 2] : 0.0;
    // Cartesian: sigma + x and y diagonals; CYL: the x diagonal is added per plane, scaled
    dxy[s] = CYL ? a.sigma[r] + cy[3 * j + 1] : a.sigma[r] + cxd + cy[3 * j + 1];
  }
  const TU* ucol = u + rbase + ic;
  auto at = [&](int k, int s) { return ucol + k * plane + static_cast<long long>(jr[s]) * a.nx; };
  // u is held in its storage type and widened where it is used, so no conversion waits for a
  // load ahead of the arithmetic
  TU um[JS], uc[JS + 2], up[JS + 2];
#pragma unroll
  for (int s = 0; s < JS; ++s) um[s] = k0 > 0 ? *at(k0 - 1, s + 1) : TU(0);
#pragma unroll
  for (int s = 0; s < JS + 2; ++s) uc[s] = *at(k0, s);
  for (int k = k0; k < k1; ++k) {
    double xs[JS], fv[JS];
    // x neighbours and f of plane k first, plane k+1 (next step's centre) last
#pragma unroll
    for (int s = 0; s < JS; ++s) {
      TU lo = lane_below(uc[s + 1], lane), hi = lane_above(uc[s + 1], lane);
      const TU* p = at(k, s + 1);
      if (lane == 0 && hx_lo && ic > 0) lo = p[-1];
      if (lane == 63 && hx_hi && ic + 1 < a.nx) hi = p[1];
      if (xper && ic == 0) lo = p[a.nx - 1];      // periodic wrap: the last column of the row
      if (xper && ic == a.nx - 1) hi = p[1 - a.nx];  // and its first
      xs[s] = (hx_lo ? cxl * static_cast<double>(lo) : 0.0) + (hx_hi ? cxu * static_cast<double>(hi) : 0.0);
      fv[s] = MODE == 1 ? f[rbase + k * plane + static_cast<long long>(jr[s + 1]) * a.nx + ic] : 0.0;
    }
    const bool has_up = k + 1 < a.nz;
#pragma unroll
    for (int s = 0; s < JS + 2; ++s) up[s] = has_up ? *at(k + 1, s) : TU(0);
    const double czl = cz[3 * k], czd = cz[3 * k + 1], czu = cz[3 * k + 2];
    const double xsk = CYL ? a.xscale[k] : 1.0;
#pragma unroll
    for (int s = 0; s < JS; ++s) {
      const double dd = CYL ? dxy[s] + czd + xsk * cxd : dxy[s] + czd;
      const double xt = CYL ? xsk * xs[s] : xs[s];
      const double h = dd * static_cast<double>(uc[s + 1]) + czl * static_cast<double>(um[s]) +
                       czu * static_cast<double>(up[s + 1]) + cyl[s] * static_cast<double>(uc[s]) +
                       cyu[s] * static_cast<double>(uc[s + 2]) + xt;
      const double res = MODE == 1 ? fv[s] - h : h;
      if (iok && j0 + s < a.ny) out[rbase + k * plane + static_cast<long long>(j0 + s) * a.nx + i] = store_cvt<TOut>(res);
    }
#pragma unroll
    for (int s = 0; s < JS; ++s) um[s] = uc[s + 1];
#pragma unroll
    for (int s = 0; s < JS + 2; ++s) uc[s] = up[s];
  }
}

template <typename TOut>
__global__ __launch_bounds__(256) void k_convert(const double* __restrict__ f, TOut* __restrict__ out, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = store_cvt<TOut>(f[i]);
}

namespace {
template <typename TU>
hipError_t stencil_any(int mode, const TU* u, const double* f, void* out, Prec tout, const StencilArgs& a,
                       hipStream_t st) {
  const long long n = static_cast<long long>(a.nx) * a.ny * a.nz * a.nrhs;
  if (n == 0) return hipSuccess;
  // the cylindrical operator is built for FP64 u and output only, and is never grouped
  if (a.xscale && (mode == 2 || !std::is_same<TU, double>::value || tout != P_F64 || a.cx_rhs))
    return hipErrorInvalidValue;
  if (!a.cx_rhs != !a.cy_rhs || !a.cx_rhs != !a.cz_rhs) return hipErrorInvalidValue;
  if (mode == 2) {
    const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
    if (tout == P_F64)
      hipLaunchKernelGGL(k_convert<double>, grid, block, 0, st, f, static_cast<double*>(out), n);
    else if (tout == P_F32)
      hipLaunchKernelGGL(k_convert<float>, grid, block, 0, st, f, static_cast<float*>(out), n);
    else
      hipLaunchKernelGGL(k_convert<bf16_t>, grid, block, 0, st, f, static_cast<bf16_t*>(out), n);
    return hipGetLastError();
  }
  // waves side by side in x: 4 for nx > 128, 2 for nx > 64, else 1 (the rest stack in y)
  const int wx = a.nx > 128 ? 4 : (a.nx > 64 ? 2 : 1);
  const int nbx = (a.nx + 64 * wx - 1) / (64 * wx);
  const int rows = (4 / wx) * kStencilJS;  // y rows per workgroup
  const int nby = (a.ny + rows - 1) / rows;
  const long long xy_blocks = static_cast<long long>(nbx) * nby * a.nrhs;
  // z-chunks: enough workgroups to fill the chip (about 4096), chunks of at least 4 planes
  int nzc = static_cast<int>(std::max<long long>(1, std::min<long long>((a.nz + 3) / 4, (4096 + xy_blocks - 1) / xy_blocks)));
  const int zchunk = (a.nz + nzc - 1) / nzc;
  nzc = (a.nz + zchunk - 1) / zchunk;
  const long long tiles = xy_blocks * nzc;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(tiles)), block(256);
  auto launch = [&](auto out_type, auto mode_c) {
    using TOut = decltype(out_type);
    if constexpr (std::is_same<TU, double>::value && std::is_same<TOut, double>::value) {
      if (a.xscale) {  // cylindrical plans: FP64 operator and residual only
        hipLaunchKernelGGL((k_stencil<TOut, decltype(mode_c)::value, TU, true>), grid, block, 0, st, u, f,
                           static_cast<TOut*>(out), a, zchunk, nzc, wx, nbx, nby);
        return;
      }
    }
    hipLaunchKernelGGL((k_stencil<TOut, decltype(mode_c)::value, TU>), grid, block, 0, st, u, f,
                       static_cast<TOut*>(out), a, zchunk, nzc, wx, nbx, nby);
  };
  using M0 = std::integral_constant<int, 0>;
  using M1 = std::integral_constant<int, 1>;
  if (tout == P_F64)
    mode == 1 ? launch(double{}, M1{}) : launch(double{}, M0{});
  else if (tout == P_F32)
    mode == 1 ? launch(float{}, M1{}) : launch(float{}, M0{});
  else
    mode == 1 ? launch(bf16_t{}, M1{}) : launch(bf16_t{}, M0{});
  return hipGetLastError();
}
}  // namespace

hipError_t stencil(int mode, const double* u, const double* f, void* out, Prec tout, const StencilArgs& a,
                   hipStream_t st) {
  return stencil_any(mode, u, f, out, tout, a, st);
}

hipError_t stencil_u32(int mode, const float* u, const double* f, void* out, Prec tout, const StencilArgs& a,
                       hipStream_t st) {
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  return stencil_any(mode, u, f, out, tout, a, st);
}

// ------------------------------------------------------------------ refinement update
// Grid-stride over the points of one RHS (blockIdx.y); each lane updates 4 consecutive points
// per step (16-byte FP32 load, two 16-byte FP64 load/stores).  Norms: wave max, then a block
// max through LDS, then one striped atomic pair per workgroup.  SRC: the value d is added to:
// 0 the FP64 u in place, 1 nothing (u = d), 2 an FP32 first solve u0 (u = u0 + d).
template <int SRC>
__global__ __launch_bounds__(256) void k_update(double* __restrict__ u, const float* __restrict__ d,
                                                const float* __restrict__ u0, long long P,
                                                unsigned long long* __restrict__ norms) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  __shared__ double sh[2][4];
  __shared__ int shbad[4];
  const int r = blockIdx.y;
  double* ur = u + r * P;
  const float* dr = d + r * P;
  const float* u0r = SRC == 2 ? u0 + r * P : nullptr;
  double dm = 0.0, um = 0.0;
  bool bad = false;
  const long long stride = static_cast<long long>(gridDim.x) * 1024;
  for (long long i0 = (static_cast<long long>(blockIdx.x) * 256 + threadIdx.x) * 4; i0 < P; i0 += stride) {
    if (i0 + 3 < P && (P & 3) == 0) {
      const f4 dv = *reinterpret_cast<const f4*>(dr + i0);
      d2v a = d2v{0, 0}, b = d2v{0, 0};
      if constexpr (SRC == 0) {
        a = *reinterpret_cast<const d2v*>(ur + i0);
        b = *reinterpret_cast<const d2v*>(ur + i0 + 2);
      } else if constexpr (SRC == 2) {
        const f4 ov = *reinterpret_cast<const f4*>(u0r + i0);
        a = d2v{static_cast<double>(ov[0]), static_cast<double>(ov[1])};
        b = d2v{static_cast<double>(ov[2]), static_cast<double>(ov[3])};
      }
      a[0] += dv[0];
      a[1] += dv[1];
      b[0] += dv[2];
      b[1] += dv[3];
      *reinterpret_cast<d2v*>(ur + i0) = a;
      *reinterpret_cast<d2v*>(ur + i0 + 2) = b;
      const double m1 = fmax(fmax(fabs(static_cast<double>(dv[0])), fabs(static_cast<double>(dv[1]))),
                             fmax(fabs(static_cast<double>(dv[2])), fabs(static_cast<double>(dv[3]))));
      const double m2 = fmax(fmax(fabs(a[0]), fabs(a[1])), fmax(fabs(b[0]), fabs(b[1])));
      bad = bad || !(m1 == m1) || !(m2 == m2);
      dm = fmax(dm, m1);
      um = fmax(um, m2);
    } else {
      for (long long i = i0; i < i0 + 4 && i < P; ++i) {
        const double dv = dr[i];
        const double old = SRC == 0 ? ur[i] : (SRC == 2 ? static_cast<double>(u0r[i]) : 0.0);
        const double un = old + dv;
        ur[i] = un;
        bad = bad || !(dv == dv) || !(un == un);
        dm = fmax(dm, fabs(dv));
        um = fmax(um, fabs(un));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    dm = fmax(dm, __shfl_xor(dm, o));
    um = fmax(um, __shfl_xor(um, o));
  }
  const int wave = threadIdx.x >> 6;
  const bool wbad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    sh[0][wave] = dm;
    sh[1][wave] = um;
    shbad[wave] = wbad ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bd = 0.0, bu = 0.0;
    int anybad = 0;
    for (int w = 0; w < 4; ++w) {
      bd = fmax(bd, sh[0][w]);
      bu = fmax(bu, sh[1][w]);
      anybad |= shbad[w];
    }
    atomic_max_nonneg(norm_slot(norms, r, 0), anybad ? __longlong_as_double(0x7ff8000000000000ll) : bd);
    atomic_max_nonneg(norm_slot(norms, r, 1), bu);
  }
}

hipError_t update_u(double* u, const float* d, long long P, int nrhs, int assign, unsigned long long* norms,
                    hipStream_t st, const float* u0) {
  if (P <= 0 || nrhs <= 0) return hipSuccess;
  // one pass of the loop per thread where the grid allows: a thread that loops issues its next
  // loads after its stores, which the in-order memory counter makes wait for those stores
  // (2048 workgroups, 8 passes at 256^3: 53 us; one pass: 49.6 us)
  const long long blocks = std::min<long long>((P + 1023) / 1024, 65535);
  const dim3 grid(static_cast<unsigned>(blocks), nrhs), block(256);
  if (u0)
    hipLaunchKernelGGL(k_update<2>, grid, block, 0, st, u, d, u0, P, norms);
  else if (assign)
    hipLaunchKernelGGL(k_update<1>, grid, block, 0, st, u, d, u0, P, norms);
  else
    hipLaunchKernelGGL(k_update<0>, grid, block, 0, st, u, d, u0, P, norms);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small helpers

// Deterministic volume-weighted sums: stage 1 writes one partial per block, stage 2 sums
// them in a fixed order, stage 3 subtracts the mean.
// Volume-weighted sum, deterministic: workgroup g of a RHS takes the x-rows q = g, g + G, ...
// (q = k * ny + j, weight vz[k] vy[j] per row) with its lanes striding the row, then a fixed
// tree in LDS; the G partials are summed by one workgroup in a fixed tree as well.
__global__ __launch_bounds__(256) void k_wsum_partial(const double* __restrict__ x, const double* __restrict__ vx,
                                                      const double* __restrict__ vy, const double* __restrict__ vz,
                                                      int nx, int ny, int nz, int blocks_per_rhs,
                                                      double* __restrict__ part) {
  __shared__ double sh[256];
  const int r = blockIdx.y;
  const long long P = static_cast<long long>(nx) * ny * nz;
  const double* xr = x + r * P;
  const int rows = ny * nz;
  double s = 0.0;
#pragma unroll 4
  for (int q = blockIdx.x; q < rows; q += blocks_per_rhs) {
    const int c = q / ny, b = q - c * ny;
    const double* row = xr + static_cast<long long>(q) * nx;
    double t = 0.0;
    for (int a = threadIdx.x; a < nx; a += 256) t += vx[a] * row[a];
    s += vz[c] * vy[b] * t;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[static_cast<long long>(r) * blocks_per_rhs + blockIdx.x] = sh[0];
}
__global__ __launch_bounds__(256) void k_wsum_final(const double* __restrict__ part, int blocks_per_rhs,
                                                    double inv_volsum, double* __restrict__ mean) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < blocks_per_rhs; i += 256) s += part[static_cast<long long>(r) * blocks_per_rhs + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[r] = sh[0] * inv_volsum;
}
__global__ __launch_bounds__(256) void k_sub_mean(double* x, const double* mean, long long P,
                                                  unsigned long long mask) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= P || !((mask >> r) & 1ull)) return;
  x[r * P + i] -= mean[r];
}

hipError_t remove_mean(double* x, const double* volx, const double* voly, const double* volz, int nx, int ny, int nz,
                       int nrhs, double inv_volsum, unsigned long long mask, double* scratch, hipStream_t st) {
  // scratch: at least nrhs * (kMeanBlocks + 1) doubles
  double* part = scratch;
  double* mean = scratch + static_cast<long long>(nrhs) * kMeanBlocks;
  hipLaunchKernelGGL(k_wsum_partial, dim3(kMeanBlocks, nrhs), dim3(256), 0, st, x, volx, voly, volz, nx, ny, nz,
                     kMeanBlocks, part);
  hipLaunchKernelGGL(k_wsum_final, dim3(nrhs), dim3(256), 0, st, part, kMeanBlocks, inv_volsum, mean);
  const long long P = static_cast<long long>(nx) * ny * nz;
  hipLaunchKernelGGL(k_sub_mean, dim3(static_cast<unsigned>((P + 255) / 256), nrhs), dim3(256), 0, st, x, mean, P,
                     mask);
  return hipGetLastError();
}

// ------------------------------------------------------------------ MAC grad / div (pressure matrix)
// 3D launch over (x, y, z) of the output grid: no index division.
__global__ __launch_bounds__(256) void k_mac_grad(int d, const double* __restrict__ p, double* __restrict__ v, int nx,
                                                  int ny, int nz, const double* __restrict__ inv_dc) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  int vx = nx, vy = ny;
  if (d == 0) vx = nx - 1;
  if (d == 1) vy = ny - 1;
  const int vz = d == 2 ? nz - 1 : nz;
  if (i >= vx || j >= vy || k >= vz) return;
  const long long pidx = (static_cast<long long>(k) * ny + j) * nx + i;
  const long long step = d == 0 ? 1 : (d == 1 ? nx : static_cast<long long>(nx) * ny);
  const int c = d == 0 ? i : (d == 1 ? j : k);
  v[(static_cast<long long>(k) * vy + j) * vx + i] = (p[pidx + step] - p[pidx]) * inv_dc[c];
}

__global__ __launch_bounds__(256) void k_mac_div_acc(int d, const double* __restrict__ v, double* __restrict__ y,
                                                     int nx, int ny, int nz, const double* __restrict__ inv_w,
                                                     double alpha) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  if (i >= nx || j >= ny || k >= nz) return;
  int vx = nx, vy = ny;
  if (d == 0) vx = nx - 1;
  if (d == 1) vy = ny - 1;
  const int c = d == 0 ? i : (d == 1 ? j : k);
  const int nd = d == 0 ? nx : (d == 1 ? ny : nz);
  const long long vidx = (static_cast<long long>(k) * vy + j) * vx + i;  // face above the cell (node c)
  const long long step = d == 0 ? 1 : (d == 1 ? vx : static_cast<long long>(vx) * vy);
  const double hi = c < nd - 1 ? v[vidx] : 0.0;
  const double lo = c > 0 ? v[vidx - step] : 0.0;
  y[(static_cast<long long>(k) * ny + j) * nx + i] += alpha * (hi - lo) * inv_w[c];
}

hipError_t mac_grad(int d, const double* p, double* v, const int n[3], const double* inv_dc, hipStream_t st) {
  const int vz = d == 2 ? n[2] - 1 : n[2];
  const dim3 grid((n[0] + 63) / 64, (n[1] + 3) / 4, vz), block(64, 4);
  hipLaunchKernelGGL(k_mac_grad, grid, block, 0, st, d, p, v, n[0], n[1], n[2], inv_dc);
  return hipGetLastError();
}

hipError_t mac_div_acc(int d, const double* v, double* y, const int n[3], const double* inv_w, double alpha,
                       hipStream_t st) {
  const dim3 grid((n[0] + 63) / 64, (n[1] + 3) / 4, n[2]), block(64, 4);
  hipLaunchKernelGGL(k_mac_div_acc, grid, block, 0, st, d, v, y, n[0], n[1], n[2], inv_w, alpha);
  return hipGetLastError();
}

__global__ void k_fill(double* y, long long n, double value) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = value;
}
hipError_t fill(double* y, long long n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, y, n, value);
  return hipGetLastError();
}

// Krylov-basis reductions and updates of FGMRES.  Both stream the basis once per call: a
// thread reads its slice of w (or its outputs) once for up to kDotVec basis vectors, with
// 16-byte loads when every row is 16-byte aligned (VW = 2) and 8-byte loads otherwise.
constexpr int kDotVec = 16;
template <int VW>
struct DotVec;
template <>
struct DotVec<1> {
  typedef double T;
  __device__ static double dot(T a, T b) { return a * b; }
};
template <>
struct DotVec<2> {
  typedef double T __attribute__((ext_vector_type(2)));
  __device__ static double dot(T a, T b) { return a.x * b.x + a.y * b.y; }
};

// Stage 1: block b sums its grid-strided slice of V_j . w for the NV vectors V_0 .. V_{NV-1}
// of this launch into partial[j][b] (fixed order: deterministic).  NV is a template
// parameter so that no load is guarded: a guarded load would end its own basic block and the
// wait at the join would serialize the loads.
template <int VW, int NV>
__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V, long long ldv,
                                                  const double* __restrict__ w, long long n,
                                                  double* __restrict__ partial) {
  typedef typename DotVec<VW>::T T;
  __shared__ double sh[4][NV];
  const long long nq = n / VW;  // VW = 2 only when n is even
  const T* wq = reinterpret_cast<const T*>(w);
  double s[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) s[j] = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x; i < nq;
       i += static_cast<long long>(gridDim.x) * 256) {
    const T wv = wq[i];
    T v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = reinterpret_cast<const T*>(V + j * ldv)[i];
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] += DotVec<VW>::dot(v[j], wv);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double v = s[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sh[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV)
    partial[static_cast<long long>(threadIdx.x) * gridDim.x + blockIdx.x] =
        (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}
// Stage 2: one block per vector sums its partials in a fixed tree order.
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int nblk,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[static_cast<long long>(j) * nblk + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}

namespace {
bool rows16(const void* p, long long ldv, long long n) {
  return reinterpret_cast<uintptr_t>(p) % 16 == 0 && ldv % 2 == 0 && n % 2 == 0;
}
}  // namespace

namespace {
template <int VW, int NV>
void launch_multidot(const double* V, long long ldv, const double* w, long long n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL((k_multidot<VW, NV>), dim3(kDotBlocks), dim3(256), 0, st, V, ldv, w, n, partial);
}
// one launch for nv (1 .. kDotVec) vectors
template <int VW>
void multidot_chunk(int nv, const double* V, long long ldv, const double* w, long long n, double* partial,
                    hipStream_t st) {
  switch (nv) {
#define HELM_DOT_CASE(k) \
  case k: launch_multidot<VW, k>(V, ldv, w, n, partial, st); break;
    HELM_DOT_CASE(1) HELM_DOT_CASE(2) HELM_DOT_CASE(3) HELM_DOT_CASE(4) HELM_DOT_CASE(5) HELM_DOT_CASE(6)
    HELM_DOT_CASE(7) HELM_DOT_CASE(8) HELM_DOT_CASE(9) HELM_DOT_CASE(10) HELM_DOT_CASE(11) HELM_DOT_CASE(12)
    HELM_DOT_CASE(13) HELM_DOT_CASE(14) HELM_DOT_CASE(15) HELM_DOT_CASE(16)
#undef HELM_DOT_CASE
    default: break;
  }
}
}  // namespace

hipError_t multi_dot(const double* V, long long ldv, int nvec, const double* w, long long n, double* partial,
                     double* out, hipStream_t st) {
  if (nvec <= 0) return hipSuccess;
  static_assert(kDotVec == 16, "multidot_chunk instantiates 1 .. 16 vectors");
  const bool v2 = rows16(V, ldv, n) && reinterpret_cast<uintptr_t>(w) % 16 == 0;
  for (int j0 = 0; j0 < nvec; j0 += kDotVec) {
    const int nv = std::min(kDotVec, nvec - j0);
    double* pj = partial + static_cast<long long>(j0) * kDotBlocks;
    if (v2)
      multidot_chunk<2>(nv, V + j0 * ldv, ldv, w, n, pj, st);
    else
      multidot_chunk<1>(nv, V + j0 * ldv, ldv, w, n, pj, st);
  }
  hipLaunchKernelGGL(k_sum_partials, dim3(nvec), dim3(256), 0, st, partial, kDotBlocks, out);
  return hipGetLastError();
}

// w[i] += sum_j coef[j] V_j[i] for the NV vectors of the basis, then the projections V_j . w and
// |w|^2 of the updated w, in one sweep: each thread keeps its values of the NV vectors in
// registers between the update and the products (two points per thread, 16-byte loads).
// partial[j][b] for j < NV, partial[NV][b] = |w|^2 (fixed order: deterministic).
template <int NV>
__global__ __launch_bounds__(256) void k_axpy_dot(double* __restrict__ w, const double* __restrict__ V,
                                                  long long ldv, const double* __restrict__ coef, long long n,
                                                  double* __restrict__ partial) {
  typedef DotVec<2>::T T;
  __shared__ double sh[4][NV + 1];
  const long long nq = n / 2;
  T* wq = reinterpret_cast<T*>(w);
  double c[NV], s[NV + 1];
#pragma unroll
  for (int j = 0; j < NV; ++j) c[j] = coef[j];
#pragma unroll
  for (int j = 0; j <= NV; ++j) s[j] = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x; i < nq;
       i += static_cast<long long>(gridDim.x) * 256) {
    T v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = reinterpret_cast<const T*>(V + j * ldv)[i];
    T x = wq[i];
#pragma unroll
    for (int j = 0; j < NV; ++j) x += c[j] * v[j];
    wq[i] = x;
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] += DotVec<2>::dot(v[j], x);
    s[NV] += DotVec<2>::dot(x, x);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j <= NV; ++j) {
    double v = s[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sh[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x <= NV)
    partial[static_cast<long long>(threadIdx.x) * gridDim.x + blockIdx.x] =
        (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

namespace {
template <int NV>
void launch_axpy_dot(double* w, const double* V, long long ldv, const double* coef, long long n, double* partial,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_axpy_dot<NV>), dim3(kDotBlocks), dim3(256), 0, st, w, V, ldv, coef, n, partial);
}
template <int NV>
bool axpy_dot_upto(int nvec, double* w, const double* V, long long ldv, const double* coef, long long n,
                   double* partial, hipStream_t st) {
  if constexpr (NV > kAxpyDotMax) {
    return false;
  } else {
    if (nvec == NV) {
      launch_axpy_dot<NV>(w, V, ldv, coef, n, partial, st);
      return true;
    }
    return axpy_dot_upto<NV + 1>(nvec, w, V, ldv, coef, n, partial, st);
  }
}
}  // namespace

hipError_t multi_axpy_dot(double* w, const double* V, long long ldv, int nvec, const double* coef, long long n,
                          double* partial, double* out, hipStream_t st) {
  if (nvec < 1 || nvec > kAxpyDotMax || !rows16(V, ldv, n) || reinterpret_cast<uintptr_t>(w) % 16)
    return hipErrorInvalidValue;
  if (!axpy_dot_upto<1>(nvec, w, V, ldv, coef, n, partial, st)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum_partials, dim3(nvec + 1), dim3(256), 0, st, partial, kDotBlocks, out);
  return hipGetLastError();
}

// w[i] += sum_j coef[j] V_j[i]: each thread owns VW consecutive points and reads its values of
// every basis vector once (eight vectors per unrolled step).
template <int VW>
__global__ __launch_bounds__(256) void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V,
                                                    long long ldv, int nvec, const double* __restrict__ coef,
                                                    long long n) {
  typedef typename DotVec<VW>::T T;
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n / VW) return;
  T* wq = reinterpret_cast<T*>(w);
  T s = wq[i];
  int j = 0;
  for (; j + 8 <= nvec; j += 8) {
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = reinterpret_cast<const T*>(V + (j + q) * ldv)[i];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += coef[j + q] * v[q];
  }
  for (; j < nvec; ++j) s += coef[j] * reinterpret_cast<const T*>(V + j * ldv)[i];
  wq[i] = s;
}
hipError_t multi_axpy(double* w, const double* V, long long ldv, int nvec, const double* coef, long long n,
                      hipStream_t st) {
  if (n <= 0 || nvec <= 0) return hipSuccess;
  if (rows16(V, ldv, n) && reinterpret_cast<uintptr_t>(w) % 16 == 0)
    hipLaunchKernelGGL(k_multi_axpy<2>, dim3(static_cast<unsigned>((n / 2 + 255) / 256)), dim3(256), 0, st, w, V,
                       ldv, nvec, coef, n);
  else
    hipLaunchKernelGGL(k_multi_axpy<1>, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, w, V, ldv,
                       nvec, coef, n);
  return hipGetLastError();
}

__global__ void k_axpby(double* y, double a, const double* x, double b, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * y[i] + b * x[i];
}
hipError_t axpby(double* y, double a, const double* x, double b, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, y, a, x, b, n);
  return hipGetLastError();
}

__global__ void k_scale(double* y, const double* x, double a, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}
hipError_t scale(double* y, const double* x, double a, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}

namespace {
struct PtrBlock {
  const void* p[kPtrBlock];
};
__global__ __launch_bounds__(256) void k_write_ptrs(PtrBlock b, int n, const void** dst) {
  // vector stores of the argument block into global memory
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = b.p[i];
}
}  // namespace

hipError_t write_ptrs(const void* const* src, int n, const void** dst, hipStream_t st) {
  for (int o = 0; o < n; o += kPtrBlock) {
    PtrBlock b{};
    const int m = n - o < kPtrBlock ? n - o : kPtrBlock;
    for (int i = 0; i < m; ++i) b.p[i] = src[o + i];
    hipLaunchKernelGGL(k_write_ptrs, dim3(1), dim3(256), 0, st, b, m, dst + o);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace helm
