// Fast sine/cosine transforms for uniform axes (the O(N log N) route the paper names for
// uniform grids in Section 1 and Section 3's operation counts).
//
// On a uniform axis the eigenvectors of the 1D operator are sampled sines or cosines
//     phi_k(j) = trig(pi (k + alpha)(j + beta) / M),
// with (trig, alpha, beta, M) fixed by the node location and the walls (DST-II, DCT-II, DST-IV,
// DCT-IV, DST-I).  The forward transform g_k = (1/nu_k) sum_j x_j phi_k(j) (nu_k = sum_j
// phi_k(j)^2, so that it is E^{-1}) and the inverse u_j = sum_k y_k phi_k(j) (E) are both
//     out_p = Re( post_p * sum_{q < L} y_q w^{p q} ),  y_q = in_q pre_q (q < N), 0 beyond,
// one complex DFT of length L = 2M with w = e^{2 pi i / L}: pre_q = e^{i pi A q / M},
// post_p = s_p e^{i pi (p + A) B / M} (times -i for sines), (A, B) = (alpha, beta) forward and
// (beta, alpha) inverse, s_p = 1/nu_p forward and 1 inverse.  Two real lines travel in one
// complex sequence (real and imaginary part) and are separated after the DFT by its conjugate
// symmetry, so a DFT of length L serves two lines.  The DFT is a Stockham auto-sorting FFT over
// radices 2, 4, 8 (butterflies written out) and 3, 5, 7 (direct sums) in LDS, one workgroup per
// batch of lines; the tables are built on the host in extended precision.  The z-forward
// transform can end with the divide of eqs. 26-28.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "fft.hpp"
#include "mode_common.hpp"

namespace helm {

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

__device__ inline d2 cmul(d2 a, d2 b) { return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline d2 mul_i(d2 a) { return d2{-a.y, a.x}; }  // i * a

// 4-point DFT with the positive exponent (i^{pq})
__device__ __attribute__((always_inline)) inline void dft4(d2& v0, d2& v1, d2& v2, d2& v3) {
  const d2 s02 = v0 + v2, d02 = v0 - v2, s13 = v1 + v3, d13 = mul_i(v1 - v3);
  v0 = s02 + s13;
  v2 = s02 - s13;
  v1 = d02 + d13;
  v3 = d02 - d13;
}

// One Stockham stage of radix R over the B sequences of length L held in buf, Ns = product of the
// radices of the earlier stages.  Every thread gathers its butterflies, twiddles them, forms
// the R-point DFTs in registers, waits for the whole workgroup, then scatters.
template <int R>
__device__ __attribute__((always_inline)) inline void stage(d2* buf, int L, int B, int Ns, const d2* __restrict__ W) {
  constexpr int U = (kFftBuf / R + 255) / 256;
  const int nb = L / R;
  const int total = B * nb;
  const int step = L / (Ns * R);
  d2 root[R];  // odd radices: the R roots e^{2 pi i m / R}, read once
  if constexpr (R != 2 && R != 4 && R != 8) {
#pragma unroll
    for (int m = 0; m < R; ++m) root[m] = W[m * (L / R)];
  }
  d2 res[U][R];
  int dst[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = threadIdx.x + 256 * u;
    dst[u] = -1;
    if (t >= total) continue;
    const int b = t / nb, j = t - b * nb;
    const int k = j % Ns;
    d2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = buf[fft_lds_index(b * L + j + q * nb)];
    if (k != 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = cmul(v[q], W[q * k * step]);
    }
    if constexpr (R == 2) {
      res[u][0] = v[0] + v[1];
      res[u][1] = v[0] - v[1];
    } else if constexpr (R == 4) {
      dft4(v[0], v[1], v[2], v[3]);
#pragma unroll
      for (int p = 0; p < 4; ++p) res[u][p] = v[p];
    } else if constexpr (R == 8) {
      // even and odd halves, then w_p = E_{p mod 4} + e^{i pi p / 4} O_{p mod 4}
      d2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
      dft4(e0, e1, e2, e3);
      dft4(o0, o1, o2, o3);
      const double c = 0.70710678118654752440;
      const d2 t1 = d2{c * (o1.x - o1.y), c * (o1.x + o1.y)};   // e^{i pi/4} o1
      const d2 t2 = mul_i(o2);                                   // e^{i pi/2} o2
      const d2 t3 = d2{-c * (o3.x + o3.y), c * (o3.x - o3.y)};   // e^{3 i pi/4} o3
      res[u][0] = e0 + o0;
      res[u][4] = e0 - o0;
      res[u][1] = e1 + t1;
      res[u][5] = e1 - t1;
      res[u][2] = e2 + t2;
      res[u][6] = e2 - t2;
      res[u][3] = e3 + t3;
      res[u][7] = e3 - t3;
    } else {
      // odd radix: direct sum with e^{2 pi i p q / R} = root[p q mod R]
#pragma unroll
      for (int p = 0; p < R; ++p) {
        d2 acc = v[0];
#pragma unroll
        for (int q = 1; q < R; ++q) acc += cmul(v[q], root[(p * q) % R]);
        res[u][p] = acc;
      }
    }
    dst[u] = b * L + (j / Ns) * Ns * R + k;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (dst[u] >= 0) {
#pragma unroll
      for (int p = 0; p < R; ++p) buf[fft_lds_index(dst[u] + p * Ns)] = res[u][p];
    }
  __syncthreads();
}

// Two real lines share one complex sequence: z = (x + i x') pre, Z = DFT(z).  With
// Y_p = sum_q x_q w^{(p + A) q} (w = e^{2 pi i / L}; pre_q = w^{A q}; 2A an integer) and x real,
// Y_{L - 2A - p} = conj(Y_p), so Y_p = (Z_p + conj(Z_p')) / 2 and Y'_p = (Z_p - conj(Z_p')) / (2i)
// with p' = (L - 2A - p) mod L: one FFT serves both lines (the factor 1/2 is in post).
//
// Per-line set-up of a batch of B lines starting at line0 (nl of them exist): base offsets and,
// for the z-forward divide, the line's part lambda_x + lambda_y + sigma of the denominator.
template <int EPI>
__device__ __attribute__((always_inline)) inline void fft_lines_setup(const FftLines& ln, const EpiArgs& ep,
                                                                      long long line0, int nl, long long* lbase,
                                                                      double* lshift) {
  for (int b = threadIdx.x; b < nl; b += 256) {
    const long long line = line0 + b;
    const long long a0 = line % ln.n0, rest = line / ln.n0;
    const long long a1 = rest % ln.n1, a2 = rest / ln.n1;
    lbase[b] = a2 * ln.t2 + a1 * ln.t1 + a0 * ln.t0;
    // z-forward: the line is (rhs, y mode, x mode)
    if constexpr (EPI == EPI_DIVIDE) lshift[b] = ep.lamx[a0] + ep.lamy[a1] + ep.sigma[a2];
  }
}

// Load of sequence s, element q: z_q = (x_{2s}[q] + i x_{2s+1}[q]) pre_q for q < N, else 0.  A
// contiguous axis walks along the lines; a strided one walks across adjacent sequences, so the
// two lines of a sequence (adjacent in memory) and consecutive lanes read consecutive addresses.
__device__ __attribute__((always_inline)) inline d2 fft_load(const double* __restrict__ in, const FftLines& ln,
                                                             const long long* lbase, int nl, const d2* pre, int N,
                                                             int s, int q) {
  const int b = 2 * s;
  if (q >= N || b >= nl) return d2{0.0, 0.0};
  const double x = in[lbase[b] + q * ln.se];
  const double y = b + 1 < nl ? in[lbase[b + 1] + q * ln.se] : 0.0;
  const d2 pq = pre[q];
  return d2{x * pq.x - y * pq.y, x * pq.y + y * pq.x};
}

// Output p of line b from its sequence's spectrum: Re(post_p Y_p), Y the line's own transform.
__device__ __attribute__((always_inline)) inline double fft_out(const d2* buf, int L, int refl, const d2* post,
                                                                int b, int p) {
  const int base = (b >> 1) * L;
  int pc = refl - p;
  if (pc >= L) pc -= L;
  const d2 Z = buf[fft_lds_index(base + p)], C = buf[fft_lds_index(base + pc)];
  // first line: (Z + conj(C)) / 2, second: (Z - conj(C)) / (2i); the 1/2 is in post
  const d2 Y = (b & 1) ? d2{Z.y + C.y, C.x - Z.x} : d2{Z.x + C.x, Z.y - C.y};
  const d2 ps = post[p];
  return ps.x * Y.x - ps.y * Y.y;
}

// Outputs p of both lines of sequence sq (the two spectra share Z_p and Z_p'): Re(post_p Y_p)
// of the first line in v0, of the second in v1.
__device__ __attribute__((always_inline)) inline void fft_out2(const d2* buf, int L, int refl, const d2* post, int sq,
                                                               int p, double& v0, double& v1) {
  const int base = sq * L;
  int pc = refl - p;
  if (pc >= L) pc -= L;
  const d2 Z = buf[fft_lds_index(base + p)], C = buf[fft_lds_index(base + pc)];
  const d2 ps = post[p];
  v0 = ps.x * (Z.x + C.x) - ps.y * (Z.y - C.y);
  v1 = ps.x * (Z.y + C.y) - ps.y * (C.x - Z.x);
}

// ODD: the plan has radix-3, 5 or 7 stages (their direct sums need about twice the registers
// of the power-of-two butterflies, so power-of-two lengths use an instantiation without them).
template <int EPI, bool ODD>
__global__ __launch_bounds__(256) void k_fft(const double* __restrict__ in, double* __restrict__ out, FftTables t,
                                             FftLines ln, EpiArgs ep) {
  extern __shared__ d2 buf[];  // S sequences of L complex values
  __shared__ long long lbase[kFftMaxLines];
  __shared__ double lshift[EPI == EPI_DIVIDE ? kFftMaxLines : 1];
  const int L = t.L, N = t.N;
  const int B = t.lines, S = t.lines / 2;
  const long long line0 = static_cast<long long>(blockIdx.x) * B;
  const int nl = static_cast<int>(min<long long>(B, ln.nlines - line0));
  fft_lines_setup<EPI>(ln, ep, line0, nl, lbase, lshift);
  __syncthreads();
  const d2* pre = reinterpret_cast<const d2*>(t.pre);
  const d2* post = reinterpret_cast<const d2*>(t.post);
  const d2* W = reinterpret_cast<const d2*>(t.W);
  const bool contig = ln.se == 1;
  for (int idx = threadIdx.x; idx < S * L; idx += 256) {
    int sq, q;
    if (contig) {
      sq = idx / L;
      q = idx - sq * L;
    } else {
      q = idx / S;
      sq = idx - q * S;
    }
    buf[fft_lds_index(sq * L + q)] = fft_load(in, ln, lbase, nl, pre, N, sq, q);
  }
  __syncthreads();
  int Ns = 1;
  for (int st = 0; st < t.nst; ++st) {
    const int r = t.rad[st];
    if (r == 8) {
      stage<8>(buf, L, S, Ns, W);
    } else if (r == 4) {
      stage<4>(buf, L, S, Ns, W);
    } else if (r == 2) {
      stage<2>(buf, L, S, Ns, W);
    } else if constexpr (ODD) {
      if (r == 3)
        stage<3>(buf, L, S, Ns, W);
      else if (r == 5)
        stage<5>(buf, L, S, Ns, W);
      else
        stage<7>(buf, L, S, Ns, W);
    }
    Ns *= r;
  }
  // post-twiddle (scale and sine/cosine part folded in), optional divide, store
  for (int idx = threadIdx.x; idx < B * N; idx += 256) {
    int b, p;
    if (contig) {
      b = idx / N;
      p = idx - b * N;
    } else {
      p = idx / B;
      b = idx - p * B;
    }
    if (b >= nl) continue;
    double v = fft_out(buf, L, t.refl, post, b, p);
    if constexpr (EPI == EPI_DIVIDE) v = divide_den(v, ep, ep.lamz[p] + lshift[b]);  // p: the z mode (eqs. 26-28)
    out[lbase[b] + p * ln.se] = v;
  }
}

// ---- power-of-two lengths: L, the sequences per workgroup and every stage's radix and stride
// are compile-time constants, so the index arithmetic has no runtime divisions.
template <int L>
constexpr int pow2_seqs() {
  return kFftBuf / L < kFftMaxLines / 2 ? kFftBuf / L : kFftMaxLines / 2;
}

template <int R, int L, int Ns>
__device__ __attribute__((always_inline)) inline void stage_c(d2* buf, const d2* __restrict__ W) {
  constexpr int B = pow2_seqs<L>();
  constexpr int nb = L / R;
  constexpr int total = B * nb;
  constexpr int U = (total + 255) / 256;
  constexpr int step = L / (Ns * R);
  d2 res[U][R];
  int dst[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = threadIdx.x + 256 * u;
    dst[u] = -1;
    if (total % 256 != 0 && t >= total) continue;
    const int b = t / nb, j = t % nb;
    const int k = j % Ns;
    d2 v[R];
    // first radix-8 stage: inputs q >= 4 sit at positions >= L / 2, where the zero-padded
    // sequence is zero (the load phase writes only the first half)
    constexpr int RIN = (Ns == 1 && R == 8) ? 4 : R;
#pragma unroll
    for (int q = 0; q < RIN; ++q) v[q] = buf[fft_lds_index(b * L + j + q * nb)];
    if (Ns > 1 && k != 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = cmul(v[q], W[q * k * step]);
    }
    if constexpr (Ns == 1 && R == 8) {
      // 4-point DFTs of (v0, v2, 0, 0) and (v1, v3, 0, 0): y_p = a + i^p b
      const d2 ib2 = mul_i(v[2]), ib3 = mul_i(v[3]);
      const d2 e0 = v[0] + v[2], e1 = v[0] + ib2, e2 = v[0] - v[2], e3 = v[0] - ib2;
      const d2 o0 = v[1] + v[3], o1 = v[1] + ib3, o2 = v[1] - v[3], o3 = v[1] - ib3;
      const double c = 0.70710678118654752440;
      const d2 t1 = d2{c * (o1.x - o1.y), c * (o1.x + o1.y)};
      const d2 t2 = mul_i(o2);
      const d2 t3 = d2{-c * (o3.x + o3.y), c * (o3.x - o3.y)};
      res[u][0] = e0 + o0;
      res[u][4] = e0 - o0;
      res[u][1] = e1 + t1;
      res[u][5] = e1 - t1;
      res[u][2] = e2 + t2;
      res[u][6] = e2 - t2;
      res[u][3] = e3 + t3;
      res[u][7] = e3 - t3;
    } else if constexpr (R == 2) {
      res[u][0] = v[0] + v[1];
      res[u][1] = v[0] - v[1];
    } else if constexpr (R == 4) {
      dft4(v[0], v[1], v[2], v[3]);
#pragma unroll
      for (int p = 0; p < 4; ++p) res[u][p] = v[p];
    } else {
      d2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
      dft4(e0, e1, e2, e3);
      dft4(o0, o1, o2, o3);
      const double c = 0.70710678118654752440;
      const d2 t1 = d2{c * (o1.x - o1.y), c * (o1.x + o1.y)};
      const d2 t2 = mul_i(o2);
      const d2 t3 = d2{-c * (o3.x + o3.y), c * (o3.x - o3.y)};
      res[u][0] = e0 + o0;
      res[u][4] = e0 - o0;
      res[u][1] = e1 + t1;
      res[u][5] = e1 - t1;
      res[u][2] = e2 + t2;
      res[u][6] = e2 - t2;
      res[u][3] = e3 + t3;
      res[u][7] = e3 - t3;
    }
    dst[u] = b * L + (j / Ns) * Ns * R + k;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (dst[u] >= 0) {
#pragma unroll
      for (int p = 0; p < R; ++p) buf[fft_lds_index(dst[u] + p * Ns)] = res[u][p];
    }
  __syncthreads();
}

// radix 8 while at least 8 remain, then one radix-4 or radix-2 stage
template <int L, int Ns>
__device__ __attribute__((always_inline)) inline void stages_pow2(d2* buf, const d2* __restrict__ W) {
  constexpr int rem = L / Ns;
  if constexpr (rem >= 8) {
    stage_c<8, L, Ns>(buf, W);
    stages_pow2<L, Ns * 8>(buf, W);
  } else if constexpr (rem == 4) {
    stage_c<4, L, Ns>(buf, W);
  } else if constexpr (rem == 2) {
    stage_c<2, L, Ns>(buf, W);
  }
}

// CONTIG: the axis is the contiguous one (x); otherwise lines are adjacent in memory and the
// lanes walk across them, each lane stepping its own pointer (no 64-bit multiply per element).
template <int EPI, int L, bool CONTIG>
__global__ __launch_bounds__(256) void k_fft_pow2(const double* __restrict__ in, double* __restrict__ out,
                                                  FftTables t, FftLines ln, EpiArgs ep) {
  constexpr int S = pow2_seqs<L>();
  constexpr int B = 2 * S;
  constexpr int H = L / 2;  // N <= H values in, N outputs per line
  __shared__ d2 buf[fft_lds_index(S * L - 1) + 1];
  __shared__ long long lbase[B];
  __shared__ double lshift[EPI == EPI_DIVIDE ? B : 1];
  const int N = t.N;
  const long long line0 = static_cast<long long>(blockIdx.x) * B;
  const int nl = static_cast<int>(min<long long>(B, ln.nlines - line0));
  fft_lines_setup<EPI>(ln, ep, line0, nl, lbase, lshift);
  __syncthreads();
  const d2* pre = reinterpret_cast<const d2*>(t.pre);
  const d2* post = reinterpret_cast<const d2*>(t.post);
  const d2* W = reinterpret_cast<const d2*>(t.W);
  // the first half of every sequence (zeros from N to L / 2); the first stage reads nothing beyond it
  if constexpr (CONTIG) {
#pragma unroll 4
    for (int idx = threadIdx.x; idx < S * H; idx += 256) {
      const int sq = idx / H, q = idx % H;
      buf[fft_lds_index(sq * L + q)] = fft_load(in, ln, lbase, nl, pre, N, sq, q);
    }
  } else {
    constexpr int QS = 256 / S;  // elements a lane advances per pass
    const int sq = threadIdx.x % S, q0 = threadIdx.x / S;
    const int b = 2 * sq;
    const bool h0 = b < nl, h1 = b + 1 < nl;
    const long long step = static_cast<long long>(QS) * ln.se;
    const double* p0 = in + (h0 ? lbase[b] : 0) + q0 * ln.se;
    const double* p1 = in + (h1 ? lbase[b + 1] : 0) + q0 * ln.se;
#pragma unroll 4
    for (int q = q0; q < H; q += QS, p0 += step, p1 += step) {
      d2 z = d2{0.0, 0.0};
      if (q < N && h0) {
        const double x = *p0;
        const double y = h1 ? *p1 : 0.0;
        const d2 pq = pre[q];
        z = d2{x * pq.x - y * pq.y, x * pq.y + y * pq.x};
      }
      buf[fft_lds_index(sq * L + q)] = z;
    }
  }
  __syncthreads();
  stages_pow2<L, 1>(buf, W);
  // each lane finishes output p of both lines of a sequence (one read of Z_p, Z_p' and post_p)
  if constexpr (CONTIG) {
#pragma unroll 4
    for (int idx = threadIdx.x; idx < S * H; idx += 256) {
      const int sq = idx / H, p = idx % H;
      const int b = 2 * sq;
      if (p >= N || b >= nl) continue;
      double v0, v1;
      fft_out2(buf, L, t.refl, post, sq, p, v0, v1);
      if constexpr (EPI == EPI_DIVIDE) {
        const double lz = ep.lamz[p];
        v0 = divide_den(v0, ep, lz + lshift[b]);
        v1 = divide_den(v1, ep, lz + lshift[b + 1 < nl ? b + 1 : b]);
      }
      out[lbase[b] + p] = v0;
      if (b + 1 < nl) out[lbase[b + 1] + p] = v1;
    }
  } else {
    constexpr int PS = 256 / S;  // outputs a lane advances per pass
    const int sq = threadIdx.x % S, p0 = threadIdx.x / S;
    const int b = 2 * sq;
    if (b < nl) {
      const bool h1 = b + 1 < nl;
      const long long step = static_cast<long long>(PS) * ln.se;
      double* o0 = out + lbase[b] + p0 * ln.se;
      double* o1 = out + (h1 ? lbase[b + 1] : lbase[b]) + p0 * ln.se;
#pragma unroll 4
      for (int p = p0; p < N; p += PS, o0 += step, o1 += step) {
        double v0, v1;
        fft_out2(buf, L, t.refl, post, sq, p, v0, v1);
        if constexpr (EPI == EPI_DIVIDE) {
          const double lz = ep.lamz[p];
          v0 = divide_den(v0, ep, lz + lshift[b]);
          v1 = divide_den(v1, ep, lz + lshift[h1 ? b + 1 : b]);
        }
        *o0 = v0;
        if (h1) *o1 = v1;
      }
    }
  }
}

template <int EPI>
bool launch_pow2(int L, dim3 grid, const double* in, double* out, const FftTables& t, const FftLines& ln,
                 const EpiArgs& ep, hipStream_t st) {
  switch (L) {
#define HELM_FFT_CASE(LL)                                                                           \
  case LL:                                                                                          \
    if (t.lines != 2 * pow2_seqs<LL>()) return false;                                               \
    if (ln.se == 1)                                                                                 \
      hipLaunchKernelGGL((k_fft_pow2<EPI, LL, true>), grid, dim3(256), 0, st, in, out, t, ln, ep);  \
    else                                                                                            \
      hipLaunchKernelGGL((k_fft_pow2<EPI, LL, false>), grid, dim3(256), 0, st, in, out, t, ln, ep); \
    return true;
    HELM_FFT_CASE(8)
    HELM_FFT_CASE(16)
    HELM_FFT_CASE(32)
    HELM_FFT_CASE(64)
    HELM_FFT_CASE(128)
    HELM_FFT_CASE(256)
    HELM_FFT_CASE(512)
    HELM_FFT_CASE(1024)
#undef HELM_FFT_CASE
    default:
      return false;
  }
}

}  // namespace

bool fft_axis_params(const Axis1D& ax, int& sine, double& alpha, double& beta, int& M) {
  if (ax.periodic || !ax.gdiag.empty() || ax.faces.size() < 3) return false;  // cylindrical axes
  const int n = static_cast<int>(ax.faces.size()) - 1;
  const double h = (ax.faces[n] - ax.faces[0]) / n;
  for (int i = 0; i < n; ++i)
    if (std::fabs((ax.faces[i + 1] - ax.faces[i]) - h) > 1e-12 * h) return false;
  const bool lo_d = ax.bc_lo == 0, hi_d = ax.bc_hi == 0;
  if (ax.loc == 0) {  // cell-centred nodes (i + 1/2) h
    M = ax.m;
    beta = 0.5;
    if (lo_d && hi_d) {
      sine = 1;
      alpha = 1.0;
    } else if (!lo_d && !hi_d) {
      sine = 0;
      alpha = 0.0;
    } else {
      sine = lo_d ? 1 : 0;
      alpha = 0.5;
    }
    return true;
  }
  if (lo_d && hi_d) {  // face-located nodes (i + 1) h, i < n - 1
    sine = 1;
    alpha = 1.0;
    beta = 1.0;
    M = n;
    return true;
  }
  if (!lo_d && !hi_d) {  // face-located, Neumann: control volumes h, nodes as cell centres of M cells
    sine = 0;
    alpha = 0.0;
    beta = 0.5;
    M = ax.m;
    return true;
  }
  return false;
}

bool fft_plan(int sine, double alpha, double beta, int M, int N, bool forward, FftHost& h) {
  const int L = 2 * M;
  if (N < 1 || N > M || L > kFftMaxLen) return false;
  // radices: 8s, then 4s and 2s, then odd factors
  int rem = L, nst = 0;
  int rad[kFftMaxStages];
  for (int r : {8, 4, 2, 3, 5, 7})
    while (rem % r == 0) {
      if (nst == kFftMaxStages) return false;
      rad[nst++] = r;
      rem /= r;
    }
  if (rem != 1) return false;
  using R = long double;
  const R pi = 3.141592653589793238462643383279502884L;
  h.L = L;
  h.N = N;
  h.M = M;
  h.nst = nst;
  for (int s = 0; s < nst; ++s) h.rad[s] = rad[s];
  h.W.resize(2 * L);
  for (int m = 0; m < L; ++m) {
    const R a = 2 * pi * m / L;
    h.W[2 * m] = static_cast<double>(std::cos(a));
    h.W[2 * m + 1] = static_cast<double>(std::sin(a));
  }
  const R A = forward ? alpha : beta, B = forward ? beta : alpha;
  h.pre.resize(2 * N);
  h.post.resize(2 * N);
  for (int q = 0; q < N; ++q) {
    const R a = pi * A * q / M;
    h.pre[2 * q] = static_cast<double>(std::cos(a));
    h.pre[2 * q + 1] = static_cast<double>(std::sin(a));
  }
  for (int p = 0; p < N; ++p) {
    R sc = 0.5;  // the 1/2 of the two-lines-per-sequence split
    if (forward) {  // 1 / nu_p, nu_p = sum_j phi_p(j)^2
      R nu = 0;
      for (int j = 0; j < N; ++j) {
        const R arg = pi * (p + alpha) * (j + beta) / M;
        const R v = sine ? std::sin(arg) : std::cos(arg);
        nu += v * v;
      }
      sc = 0.5 / nu;
    }
    const R a = pi * (p + A) * B / M;
    R re = sc * std::cos(a), im = sc * std::sin(a);
    if (sine) {  // Im(z) = Re(-i z)
      const R t = re;
      re = im;
      im = -t;
    }
    h.post[2 * p] = static_cast<double>(re);
    h.post[2 * p + 1] = static_cast<double>(im);
  }
  h.lines = 2 * (kFftBuf / L < kFftMaxLines / 2 ? kFftBuf / L : kFftMaxLines / 2);
  // p' = L - 2A - p needs 2A integral (A = alpha forward, beta inverse: 0, 1/2 or 1)
  const R twoA = 2 * A;
  if (twoA != std::floor(twoA) || twoA < 0 || twoA > 2) return false;
  h.refl = L - static_cast<int>(twoA);
  return true;
}

hipError_t fft_axis(const double* in, double* out, const FftTables& t, const FftLines& ln, Epi epi,
                    const EpiArgs& ep, hipStream_t st) {
  if (ln.nlines <= 0) return hipSuccess;
  if (t.L < 2 || t.L > kFftMaxLen || t.lines < 2 || t.lines % 2 || t.lines > kFftMaxLines ||
      (t.lines / 2) * t.L > kFftBuf || t.N > t.L / 2 || t.refl < t.L - 2 || t.refl > t.L ||
      t.nst < 1 || t.nst > kFftMaxStages)
    return hipErrorInvalidValue;
  const long long blocks = (ln.nlines + t.lines - 1) / t.lines;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  bool odd = false;
  for (int s = 0; s < t.nst; ++s) {
    const int r = t.rad[s];
    if (r != 2 && r != 4 && r != 8 && r != 3 && r != 5 && r != 7) return hipErrorInvalidValue;
    odd = odd || (r & 1);
  }
  const size_t lds = static_cast<size_t>(fft_lds_index((t.lines / 2) * t.L - 1) + 1) * 2 * sizeof(double);
  const dim3 grid(static_cast<unsigned>(blocks)), block(256);
  if (epi != EPI_DIVIDE && epi != EPI_STORE) return hipErrorInvalidValue;
  // power-of-two lengths: the compile-time kernel
  if (!odd && (epi == EPI_DIVIDE ? launch_pow2<EPI_DIVIDE>(t.L, grid, in, out, t, ln, ep, st)
                                 : launch_pow2<EPI_STORE>(t.L, grid, in, out, t, ln, ep, st)))
    return hipGetLastError();
  if (epi == EPI_DIVIDE) {
    if (odd)
      hipLaunchKernelGGL((k_fft<EPI_DIVIDE, true>), grid, block, lds, st, in, out, t, ln, ep);
    else
      hipLaunchKernelGGL((k_fft<EPI_DIVIDE, false>), grid, block, lds, st, in, out, t, ln, ep);
  } else {
    if (odd)
      hipLaunchKernelGGL((k_fft<EPI_STORE, true>), grid, block, lds, st, in, out, t, ln, ep);
    else
      hipLaunchKernelGGL((k_fft<EPI_STORE, false>), grid, block, lds, st, in, out, t, ln, ep);
  }
  return hipGetLastError();
}

}  // namespace helm
