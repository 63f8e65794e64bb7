// Fast sine/cosine transforms along one axis of a uniform grid (fft.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <vector>

#include "kernels.hpp"
#include "setup.hpp"

namespace helm {

constexpr int kFftMaxLen = 1024;    // L = 2M: axes of up to 512 unknowns
constexpr int kFftMaxStages = 12;
constexpr int kFftBuf = 2048;       // complex values per workgroup (sequences * L); with the LDS padding
                                    // below the batch stays under 64 KB
// LDS index of element a of a batch: one 16-byte pad every 8 elements and one more every 512.
// A 16-byte access is served eight lanes at a time, conflict-free when those eight hit distinct
// 16-byte slots modulo 128 bytes: the first stage's scatter (stride 8 elements) and the
// sequence-strided loads (stride L) then land on distinct slots.
__host__ __device__ constexpr int fft_lds_index(int a) { return a + (a >> 3) + (a >> 9); }
constexpr int kFftMaxLines = 64;

// Device tables of one transform direction of one axis.
struct FftTables {
  int L = 0, N = 0, M = 0;      // DFT length 2M; N values in and out per line
  int nst = 0;                  // Stockham stages
  int rad[kFftMaxStages] = {};  // their radices (2, 4, 8, 3, 5, 7)
  int lines = 2;                // lines per workgroup: two per complex sequence, kFftBuf / L
                                // sequences (at most kFftMaxLines lines)
  int refl = 0;                 // L - 2A: output p of the second line of a pair needs p' = refl - p
  const double* W = nullptr;    // L complex: e^{2 pi i m / L}
  const double* pre = nullptr;  // N complex
  const double* post = nullptr; // N complex: scale, phase and the sine/cosine choice folded in
};

// Host copy of the tables, built in extended precision.
struct FftHost {
  int L = 0, N = 0, M = 0, nst = 0, lines = 2, refl = 0;
  int rad[kFftMaxStages] = {};
  std::vector<double> W, pre, post;
};

// Lines of a grid function along one axis: line index -> (a2, a1, a0) with a0 < n0 fastest and
// a1 < n1; the line starts at a2 t2 + a1 t1 + a0 t0 and its elements are se apart.  For the
// z-forward divide the line is (rhs, y mode, x mode): n0 = nx, n1 = ny.
struct FftLines {
  long long nlines = 0;
  long long n0 = 1, n1 = 1;
  long long t0 = 0, t1 = 0, t2 = 0;
  long long se = 1;
};

// Tables of phi_k(j) = trig(pi (k + alpha)(j + beta) / M) (trig = sin if sine), j, k < N, for
// the forward (E^{-1}, scaled by 1 / sum_j phi_k(j)^2) or inverse (E) transform.  False when
// 2M is beyond kFftMaxLen or has a prime factor above 7.
bool fft_plan(int sine, double alpha, double beta, int M, int N, bool forward, FftHost& h);

// The fast transform of a 1D operator built by build_operator_1d, if it has one: the faces
// are uniform (every width within 1e-12 of the mean) and the walls give a sine or cosine basis
// (cell-centred: DST-II for Dirichlet-Dirichlet, DCT-II Neumann-Neumann, DST-IV Dirichlet-
// Neumann, DCT-IV Neumann-Dirichlet; face-located: DST-I Dirichlet-Dirichlet, DCT-II
// Neumann-Neumann).  The basis is ordered by increasing eigenvalue, as the eigensolver's.
bool fft_axis_params(const Axis1D& ax, int& sine, double& alpha, double& beta, int& M);

// out = transform of in along the lines of `ln` (in == out allowed: a workgroup reads its whole
// batch before writing it); epi: EPI_STORE or EPI_DIVIDE (z-forward, eqs. 26-28).
hipError_t fft_axis(const double* in, double* out, const FftTables& t, const FftLines& ln, Epi epi,
                    const EpiArgs& ep, hipStream_t st);

}  // namespace helm
