// Launchers for the gfx950 kernels of the solve path.  Host code calls only these.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace helm {

// Waits for the work enqueued on `st` so far by spinning (with yields) on an event: the host
// needs refinement norms, Krylov scalars or a finished request at once, and a blocking stream
// synchronisation adds tens of microseconds of wake-up latency each time.  One event per host
// thread and device, created on first use; its default system-scope release makes device
// writes to pinned host memory visible when it completes.
hipError_t wait_stream(hipStream_t st);

// Storage / compute types of the mode products.
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 /* split BF16, FP32 storage */ };

// Epilogue of a mode product.
enum Epi : int {
  EPI_STORE = 0,   // Y = acc (converted to the output storage type)
  EPI_DIVIDE = 1,  // Y = acc / (lam_x[a] + lam_y[b] + lam_z[c] + sigma[r]) in FP64 (eqs. 26-28)
  EPI_ACCUM = 2,   // u += acc in FP64, with per-RHS max|acc| and max|u| (refinement update)
  EPI_STORE_F64 = 3  // Y = acc widened to FP64 (split-BF16 products: first solve writes u directly)
};

constexpr int kMaxRhs = 64;
// Refinement norms are accumulated with atomic max into kNormStripes slots per quantity (the
// slot is chosen by workgroup index) to avoid same-address contention; layout
// norms[(2 r + q) * kNormStripes + s], q = 0: max|du|, q = 1: max|u|, as FP64 bit patterns.
constexpr int kNormStripes = 64;

struct EpiArgs {
  const double* lamx = nullptr;   // eigenvalues of the x and y axes (divide epilogue)
  const double* lamy = nullptr;
  const double* lamz = nullptr;   // eigenvalues of the contracted (z) axis
  const double* lamxy = nullptr;  // lamx[a] + lamy[b] at pq = b * nx + a (split-BF16 divide)
  int nx = 1;                     // x extent, to split a column index into (b, a)
  int eq28 = 0;                   // zero denominator -> 1 (eq. 28) instead of projection
  unsigned long long* norms = nullptr;  // [2 * nrhs * kNormStripes] (accumulate), see kNormStripes
  long long rows_per_rhs = 1;     // rows of the x-mode matrix per RHS (accumulate)
  int accum_zero = 0;             // accumulate into zero instead of the current u
  double sigma[kMaxRhs];          // per-RHS shift
  // Grouped solve (right-hand sides of several plans of one shape in one launch): per-RHS
  // device tables of the operand and of the eigenvalue vectors, which replace Msw and the
  // pointers above; `span` is the extent of one RHS in the launch's tiled dimension (rows of
  // the right and rotating forms, columns of the left form), and every workgroup tile must lie
  // inside one RHS (the launchers refuse a tiling that does not divide span).  NULL: one plan.
  const void* const* msw_rhs = nullptr;
  const double* const* lamx_rhs = nullptr;
  const double* const* lamy_rhs = nullptr;
  const double* const* lamz_rhs = nullptr;
  const double* const* lamxy_rhs = nullptr;
  long long span = 0;
};
// Whether a tiling of `tile` rows or columns serves the launch (always, unless grouped).
inline bool group_tiles_ok(const EpiArgs& ep, long long tile) {
  return !ep.msw_rhs || (ep.span > 0 && ep.span % tile == 0);
}

// Bytes of one swizzled operand matrix (rows x k padded to the kernel's blocking).
size_t swizzled_bytes(Prec p, int K);
// Host-side swizzle of a row-major K x K matrix M (M[a][i]) into the fragment layout the
// mode-product kernels read; `out` must hold swizzled_bytes(p, K) bytes.
void swizzle_operand(Prec p, int K, const double* M, void* out);

// Left form (contraction along a strided axis):
//   Y[s][a][n] = sum_i M[a][i] X[s][i][n],  s < S, a < K, n < Nn.
hipError_t mode_left(Prec p, const void* Msw, int K, const void* X, Prec tin, void* Y, Prec tout,
                     long long S, long long Nn, Epi epi, const EpiArgs& ep, hipStream_t st);

// Right form (contraction along the contiguous axis):
//   Y[m][a] = sum_i X[m][i] M[a][i],  m < Mrows, a < K.
hipError_t mode_right(Prec p, const void* Msw, int K, const void* X, Prec tin, void* Y, Prec tout,
                      long long Mrows, Epi epi, const EpiArgs& ep, hipStream_t st);

// Split-BF16 rotating-layout product (three bfloat16 pieces, six MFMA partial products,
// FP32 accumulation and storage):  Y[r][a][pq] = sum_k M[a][k] X[r][pq][k],
// r < R, pq < PQ, a < K.  Msw holds the three swizzled pieces of M, `piece` elements apart.
// epi: STORE (FP32 Y), DIVIDE (FP32 Y, pq = b * nx + a_x, column a = the z index c, FP32
// divide by the FP64-summed eigenvalues, ep.lamxy required) or STORE_F64 (FP64 Y).
size_t swizzled_bf16x3_bytes(int K);
void swizzle_bf16x3(int K, const double* M, void* out);
// x_f64: X is FP64 (the solve's right-hand side, rounded to FP32 on load), else FP32.
hipError_t mode_rot(const void* Msw, int K, const void* X, bool x_f64, void* Y, long long R, long long PQ, Epi epi,
                    const EpiArgs& ep, hipStream_t st);

// Batched Thomas solve along z (TPT, end of Section 3): for every RHS r and (b, a) line,
// (K_z + c V_z) v = V_z g with c = lam_x[a] + lam_y[b] + sigma[r], in place on v (FP64).
// The line (0, 0) is skipped when skip_null != 0.  chk: scratch of thomas_scratch_bytes.
// Cylindrical plans (Section 6, eq. 44; x = theta, y = z, z = r): gdiag = dr / rc on the
// radial axis, and the line (a, b) solves (K_r + lam_theta[a] G + (lam_z[b] + sigma) V_r) v =
// V_r g with G = diag(gdiag) (NULL for Cartesian plans: G = V).
struct ThomasArgs {
  const double* kdiag;   // K_z diagonal [nz]
  const double* koff;    // K_z off-diagonal [nz - 1]
  const double* vol;     // V_z [nz]
  const double* lamx;
  const double* lamy;
  const double* gdiag = nullptr;
  int nx, ny, nz, nrhs;
  int skip_null;
  double sigma[kMaxRhs];
};
size_t thomas_scratch_bytes(int nx, int ny, int nz, int nrhs);
hipError_t thomas_z(double* v, const ThomasArgs& a, void* chk, hipStream_t st);

// The one singular z line of an all-Neumann Laplace TPT solve: v = E_z diag(1/lam') E_z^{-1} g
// on the (0, 0) line of every RHS, with 1/lam'_0 = 0 (projection) or 1 (eq. 28).  scratch:
// nrhs * nz doubles of device memory.
hipError_t null_line_z(double* v, const double* Ez, const double* Ezinv, const double* lamz, int nx, int ny, int nz,
                       int nrhs, int eq28, double* scratch, hipStream_t st);

// 7-point FP64 operator (Kronecker sum of the 1D rows plus sigma):
//   mode 0: out = H u;  mode 1: out = f - H u (residual);  mode 2: out = f (u unused);
//   stored as `tout`.
struct StencilArgs {
  const double* cx;   // [3 * nx]: lower, diag, upper rows of A_x
  const double* cy;   // [3 * ny]
  const double* cz;   // [3 * nz]
  int nx, ny, nz, nrhs;
  // Cylindrical plans (x = theta, y = z, z = r): the x term of plane k is scaled by xscale[k]
  // (1 / rc_k^2, the metric of eq. 41), and xper != 0 closes x periodically (cx's first lower
  // and last upper entries couple to the other end).  xscale NULL: Cartesian.
  const double* xscale = nullptr;
  int xper = 0;
  // Grouped solve: per-RHS device tables of cx, cy, cz (NULL: the pointers above for all RHS).
  const double* const* cx_rhs = nullptr;
  const double* const* cy_rhs = nullptr;
  const double* const* cz_rhs = nullptr;
  double sigma[kMaxRhs];
  // optional: the first workgroup clears these words (the refinement norms of the sweep the
  // residual starts), so no launch of its own is needed
  unsigned long long* zero = nullptr;
  int nzero = 0;
};
hipError_t stencil(int mode, const double* u, const double* f, void* out, Prec tout,
                   const StencilArgs& a, hipStream_t st);
// Modes 0 and 1 with u stored in FP32 (each value is exact in FP64 once read).
hipError_t stencil_u32(int mode, const float* u, const double* f, void* out, Prec tout, const StencilArgs& a,
                       hipStream_t st);

// Refinement update u += d (u = d when assign != 0; u = u0 + d when u0, an FP32 first solve,
// is given) for nrhs fields of P points, d FP32, with per-RHS max|d| and max|u| (bit patterns,
// atomic max) into norms[2 r], norms[2 r + 1].
hipError_t update_u(double* u, const float* d, long long P, int nrhs, int assign, unsigned long long* norms,
                    hipStream_t st, const float* u0 = nullptr);
// Volume-weighted mean removal per RHS: x -= sum(vol * x) * inv_volsum   (FP64, in place,
// deterministic order).  scratch: nrhs * (kMeanBlocks + 1) doubles of device memory.
constexpr int kMeanBlocks = 1024;
// Only the RHS r with bit r of `mask` set are changed.
hipError_t remove_mean(double* x, const double* volx, const double* voly, const double* volz,
                       int nx, int ny, int nz, int nrhs, double inv_volsum, unsigned long long mask,
                       double* scratch, hipStream_t st);

// ---- staggered (MAC) operators and Krylov helpers for the pressure matrix (eqs. 4, 9) ----
// Pressure grid n = (nx, ny, nz) cells; the d-velocity grid has n[d] - 1 nodes along d.
// v = Grad_d p:  v[.., i, ..] = (p[.., i+1, ..] - p[.., i, ..]) * inv_dc[i],  i < n[d] - 1.
hipError_t mac_grad(int d, const double* p, double* v, const int n[3], const double* inv_dc, hipStream_t st);
// y += alpha * Div_d v:  y[.., i, ..] += alpha * (v[.., i, ..] - v[.., i-1, ..]) * inv_w[i], wall values 0.
hipError_t mac_div_acc(int d, const double* v, double* y, const int n[3], const double* inv_w, double alpha,
                       hipStream_t st);
// y[i] = value
hipError_t fill(double* y, long long n, double value, hipStream_t st);
// out[j] = sum_i V[j * ldv + i] * w[i] for j < nvec, deterministic two-stage reduction.
// partial: nvec * kDotBlocks doubles of device scratch; out: nvec doubles (device).
constexpr int kDotBlocks = 256;
hipError_t multi_dot(const double* V, long long ldv, int nvec, const double* w, long long n, double* partial,
                     double* out, hipStream_t st);
// One sweep of w[i] += sum_j coef[j] * V[j * ldv + i] followed by out[j] = V_j . w (j < nvec)
// and out[nvec] = |w|^2 of the updated w; nvec <= kAxpyDotMax, rows and w 16-byte aligned,
// ldv and n even (else hipErrorInvalidValue, nothing launched).  partial: (nvec + 1) *
// kDotBlocks doubles of device scratch; out: nvec + 1 doubles (device).
constexpr int kAxpyDotMax = 32;
hipError_t multi_axpy_dot(double* w, const double* V, long long ldv, int nvec, const double* coef, long long n,
                          double* partial, double* out, hipStream_t st);
// w[i] += sum_j coef[j] * V[j * ldv + i]   (coef: device array of nvec values)
hipError_t multi_axpy(double* w, const double* V, long long ldv, int nvec, const double* coef, long long n,
                      hipStream_t st);
// y[i] = a * y[i] + b * x[i]
hipError_t axpby(double* y, double a, const double* x, double b, long long n, hipStream_t st);
// y[i] = a * x[i]   (x may equal y)
hipError_t scale(double* y, const double* x, double a, long long n, hipStream_t st);

// Writes n host-given pointers into device memory dst, stream-ordered (the values travel as
// kernel arguments, kPtrBlock per launch), so a grouped solve's operand tables need no host
// staging buffer and no synchronisation.
constexpr int kPtrBlock = 240;
hipError_t write_ptrs(const void* const* src, int n, const void** dst, hipStream_t st);

}  // namespace helm
