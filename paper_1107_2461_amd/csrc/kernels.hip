// gfx950 kernels of the fast-diagonalization solve path other than the mode-product
// templates (mode_common.hpp): precision dispatch of the mode products, the batched Thomas
// solve of the TPT variant, the FP64 7-point operator/residual and small helpers.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

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

hipError_t mode_left(Prec p, const void* Msw, int K, const void* X, Prec tin, void* Y, Prec tout, long long S,
                     long long Nn, Epi epi, const EpiArgs& ep, hipStream_t st) {
  const int ci = choose_cfg(K);
  if (ci < 0 || K < 1 || S < 0 || Nn < 0 || tin != p || tout != p) return hipErrorInvalidValue;
  if (epi != EPI_STORE && epi != EPI_DIVIDE) return hipErrorInvalidValue;
  if ((S * Nn + 15) / 16 > 0x7fffffffLL) return hipErrorInvalidValue;
  if (p == P_F64) return mode_left_f64(ci, Msw, K, X, Y, S, Nn, epi, ep, st);
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
  if (p == P_F32) return mode_right_f32(ci, Msw, K, X, Y, Mrows, epi, vec, ep, st);
  return mode_right_bf16(ci, Msw, K, X, Y, Mrows, epi, vec, ep, st);
}

// ------------------------------------------------------------------ Thomas along z
// One lane per (r, b, a) line; at step k a wavefront touches 64 consecutive a of one
// z-plane (coalesced).  Forward elimination keeps only a checkpoint of (pivot, rhs) every
// SEG steps; the backward sweep recomputes one segment at a time into registers, so the
// line is read twice and written once (24 B/point) and can be updated in place.
constexpr int kSeg = 16;

size_t thomas_scratch_bytes(int nx, int ny, int nz, int nrhs) {
  const long long nseg = (nz + kSeg - 1) / kSeg;
  return static_cast<size_t>(2 * nseg) * nx * ny * nrhs * sizeof(double);
}

__global__ __launch_bounds__(256) void k_thomas(double* __restrict__ v, ThomasArgs a, double* __restrict__ chk) {
  const long long Nn = static_cast<long long>(a.nx) * a.ny;
  const long long nl = Nn * a.nrhs;
  const long long line = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (line >= nl) return;
  const int r = static_cast<int>(line / Nn);
  const long long n = line - r * Nn;
  if (a.skip_null && n == 0) return;
  const int ax = static_cast<int>(n % a.nx), by = static_cast<int>(n / a.nx);
  const double c = a.lamx[ax] + a.lamy[by] + a.sigma[r];
  double* col = v + static_cast<long long>(r) * a.nz * Nn + n;
  const int nz = a.nz;
  const int nseg = (nz + kSeg - 1) / kSeg;
  // forward sweep: beta_k = D_k - m_k Koff_{k-1}, y_k = V_k g_k - m_k y_{k-1}
  double beta = 0.0, y = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double d = a.kdiag[k] + c * a.vol[k];
    const double rhs = a.vol[k] * col[static_cast<long long>(k) * Nn];
    if (k == 0) {
      beta = d;
      y = rhs;
    } else {
      const double m = a.koff[k - 1] / beta;
      beta = d - m * a.koff[k - 1];
      y = rhs - m * y;
    }
    if ((k + 1) % kSeg == 0 && k + 1 < nz) {
      const int sgi = (k + 1) / kSeg - 1;
      chk[(2LL * sgi) * nl + line] = beta;
      chk[(2LL * sgi + 1) * nl + line] = y;
    }
  }
  // backward sweep, one segment at a time from the top
  double vnext = 0.0;
  for (int j = nseg - 1; j >= 0; --j) {
    const int k0 = j * kSeg;
    double bs[kSeg], ys[kSeg];
    if (j > 0) {
      beta = chk[(2LL * (j - 1)) * nl + line];
      y = chk[(2LL * (j - 1) + 1) * nl + line];
    }
#pragma unroll
    for (int t = 0; t < kSeg; ++t) {
      const int k = k0 + t;
      if (k < nz) {
        const double d = a.kdiag[k] + c * a.vol[k];
        const double rhs = a.vol[k] * col[static_cast<long long>(k) * Nn];
        if (k == 0) {
          beta = d;
          y = rhs;
        } else {
          const double m = a.koff[k - 1] / beta;
          beta = d - m * a.koff[k - 1];
          y = rhs - m * y;
        }
      }
      bs[t] = beta;
      ys[t] = y;
    }
#pragma unroll
    for (int t = kSeg - 1; t >= 0; --t) {
      const int k = k0 + t;
      if (k < nz) {
        const double vk = (k == nz - 1) ? ys[t] / bs[t] : (ys[t] - a.koff[k] * vnext) / bs[t];
        col[static_cast<long long>(k) * Nn] = vk;
        vnext = vk;
      }
    }
  }
}

hipError_t thomas_z(double* v, const ThomasArgs& a, void* chk, hipStream_t st) {
  const long long nl = static_cast<long long>(a.nx) * a.ny * a.nrhs;
  if (nl == 0) return hipSuccess;
  const long long blocks = (nl + 255) / 256;
  hipLaunchKernelGGL(k_thomas, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, v, a, static_cast<double*>(chk));
  return hipGetLastError();
}

// ------------------------------------------------------------------ singular z line (TPT, all-Neumann)
__global__ __launch_bounds__(256) void k_null_line(double* __restrict__ v, const double* __restrict__ Ez,
                                                   const double* __restrict__ Ezinv, const double* __restrict__ lamz,
                                                   int nx, int ny, int nz, int eq28) {
  extern __shared__ double sh[];  // 2 * nz
  double* g = sh;
  double* gh = sh + nz;
  const int r = blockIdx.x;
  const long long Nn = static_cast<long long>(nx) * ny;
  double* col = v + static_cast<long long>(r) * nz * Nn;  // line (a, b) = (0, 0)
  for (int k = threadIdx.x; k < nz; k += blockDim.x) g[k] = col[static_cast<long long>(k) * Nn];
  __syncthreads();
  for (int c = threadIdx.x; c < nz; c += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nz; ++k) s += Ezinv[static_cast<long long>(c) * nz + k] * g[k];
    const double lam = lamz[c];  // the shift of this line is lam_x(0) + lam_y(0) + sigma = 0
    gh[c] = (lam == 0.0) ? (eq28 ? s : 0.0) : s / lam;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nz; k += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nz; ++c) s += Ez[static_cast<long long>(k) * nz + c] * gh[c];
    col[static_cast<long long>(k) * Nn] = s;
  }
}

hipError_t null_line_z(double* v, const double* Ez, const double* Ezinv, const double* lamz, int nx, int ny, int nz,
                       int nrhs, int eq28, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_null_line, dim3(nrhs), dim3(256), 2 * nz * sizeof(double), st, v, Ez, Ezinv, lamz, nx, ny, nz,
                     eq28);
  return hipGetLastError();
}

// ------------------------------------------------------------------ 7-point operator / residual
template <typename TOut>
__global__ __launch_bounds__(256) void k_stencil(int mode, const double* __restrict__ u, const double* __restrict__ f,
                                                 TOut* __restrict__ out, StencilArgs a) {
  const long long P = static_cast<long long>(a.nx) * a.ny * a.nz;
  const long long idx = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= P * a.nrhs) return;
  if (mode == 2) {  // plain conversion of f (the residual of u = 0)
    out[idx] = store_cvt<TOut>(f[idx]);
    return;
  }
  long long t = idx;
  const int i = static_cast<int>(t % a.nx);
  t /= a.nx;
  const int j = static_cast<int>(t % a.ny);
  t /= a.ny;
  const int k = static_cast<int>(t % a.nz);
  const int r = static_cast<int>(t / a.nz);
  const long long sy = a.nx, sz = static_cast<long long>(a.nx) * a.ny;
  const double uc = u[idx];
  double h = (a.sigma[r] + a.cx[3 * i + 1] + a.cy[3 * j + 1] + a.cz[3 * k + 1]) * uc;
  if (i > 0) h += a.cx[3 * i] * u[idx - 1];
  if (i + 1 < a.nx) h += a.cx[3 * i + 2] * u[idx + 1];
  if (j > 0) h += a.cy[3 * j] * u[idx - sy];
  if (j + 1 < a.ny) h += a.cy[3 * j + 2] * u[idx + sy];
  if (k > 0) h += a.cz[3 * k] * u[idx - sz];
  if (k + 1 < a.nz) h += a.cz[3 * k + 2] * u[idx + sz];
  const double res = mode == 1 ? f[idx] - h : h;
  out[idx] = store_cvt<TOut>(res);
}

hipError_t stencil(int mode, const double* u, const double* f, void* out, Prec tout, const StencilArgs& a,
                   hipStream_t st) {
  const long long n = static_cast<long long>(a.nx) * a.ny * a.nz * a.nrhs;
  if (n == 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  if (tout == P_F64)
    hipLaunchKernelGGL(k_stencil<double>, grid, block, 0, st, mode, u, f, static_cast<double*>(out), a);
  else if (tout == P_F32)
    hipLaunchKernelGGL(k_stencil<float>, grid, block, 0, st, mode, u, f, static_cast<float*>(out), a);
  else
    hipLaunchKernelGGL(k_stencil<bf16_t>, grid, block, 0, st, mode, u, f, static_cast<bf16_t*>(out), a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ small helpers
__global__ void k_zero_u64(unsigned long long* p, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}
hipError_t zero_u64(unsigned long long* p, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// Deterministic volume-weighted sums: stage 1 writes one partial per block, stage 2 sums
// them in a fixed order, stage 3 subtracts the mean.
__global__ __launch_bounds__(256) void k_wsum_partial(const double* __restrict__ x, const double* __restrict__ vx,
                                                      const double* __restrict__ vy, const double* __restrict__ vz,
                                                      int nx, int ny, int nz, int blocks_per_rhs,
                                                      double* __restrict__ part) {
  __shared__ double sh[256];
  const int r = blockIdx.y;
  const long long P = static_cast<long long>(nx) * ny * nz;
  const double* xr = x + r * P;
  double s = 0.0;
  for (long long i = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x; i < P;
       i += static_cast<long long>(blocks_per_rhs) * 256) {
    const int a = static_cast<int>(i % nx);
    const long long t = i / nx;
    const int b = static_cast<int>(t % ny);
    const int c = static_cast<int>(t / ny);
    s += vz[c] * vy[b] * vx[a] * xr[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[static_cast<long long>(r) * blocks_per_rhs + blockIdx.x] = sh[0];
}
__global__ void k_wsum_final(double* part, int blocks_per_rhs, double inv_volsum, double* mean) {
  const int r = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < blocks_per_rhs; ++i) s += part[static_cast<long long>(r) * blocks_per_rhs + i];
    mean[r] = s * inv_volsum;
  }
}
__global__ __launch_bounds__(256) void k_sub_mean(double* x, const double* mean, long long P, int nrhs) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= P * nrhs) return;
  x[i] -= mean[i / P];
}

hipError_t remove_mean(double* x, const double* volx, const double* voly, const double* volz, int nx, int ny, int nz,
                       int nrhs, double inv_volsum, double* scratch, hipStream_t st) {
  // scratch: at least nrhs * (kMeanBlocks + 1) doubles
  double* part = scratch;
  double* mean = scratch + static_cast<long long>(nrhs) * kMeanBlocks;
  hipLaunchKernelGGL(k_wsum_partial, dim3(kMeanBlocks, nrhs), dim3(256), 0, st, x, volx, voly, volz, nx, ny, nz,
                     kMeanBlocks, part);
  hipLaunchKernelGGL(k_wsum_final, dim3(nrhs), dim3(64), 0, st, part, kMeanBlocks, inv_volsum, mean);
  const long long P = static_cast<long long>(nx) * ny * nz;
  hipLaunchKernelGGL(k_sub_mean, dim3(static_cast<unsigned>((P * nrhs + 255) / 256)), dim3(256), 0, st, x, mean, P,
                     nrhs);
  return hipGetLastError();
}

}  // namespace helm
