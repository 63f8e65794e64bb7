// Pressure matrix of the Stokes-operator factorization and its Krylov inverse.
//
// Section 2, eq. 9: C = sum_d Grad-to-div products through the inverse velocity Helmholtz
// operators.  With the library's positive Helmholtz form H_d = (1/tau) I - Lap_h on the
// d-velocity grid of a MAC (staggered) mesh, the paper's C (written there with
// H = Lap - I/dt) is
//     C p = - sum_d Div_d H_d^{-1} Grad_d p,
// one action costing three velocity solves (the Section 2 remark on the cost of C).  The
// pressure gradient uses no pressure boundary value and the velocities are zero on the
// walls, so C annihilates constants and maps onto volume-weighted-mean-free fields.
// For small tau, H_d ~ I / tau and C ~ tau * (-Div Grad) (the Chorin limit), so the
// inverse pressure Laplacian (an all-Neumann fast-diagonalization solve) preconditions C
// (option 1, the paper's choice).  Far from that limit (1/tau below the Laplacian's large
// eigenvalues) C tends to the identity on mean-free fields instead; option 2 uses
// M^{-1} = I + (1/tau) A_p^{-1} (Cahouet & Chabard 1988), which tends to option 1 as tau -> 0
// and to the identity as tau -> infinity.
// The preconditioned Krylov iteration is flexible GMRES(m) with right preconditioning
// (the preconditioner may be an inexact, refined low-precision solve), classical
// Gram-Schmidt with one re-orthogonalization, Givens rotations on the host in FP64.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "../../include/helm.h"
#include "alloc.hpp"
#include "kernels.hpp"

using namespace helm;

namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
helm_status st_from(hipError_t e) {
  if (e == hipSuccess) return HELM_OK;
  return e == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EDEVICE;
}
}  // namespace

struct helm_pmat {
  int n[3] = {0, 0, 0};       // pressure cells
  long long np = 0;           // pressure unknowns
  long long nv[3] = {0, 0, 0};
  double tau = 0.0;
  helm_plan* vel[3] = {nullptr, nullptr, nullptr};
  helm_plan* pres = nullptr;
  size_t vel_ws = 0, pres_ws = 0;
  double* inv_dc[3] = {nullptr, nullptr, nullptr};  // 1 / (c_{i+1} - c_i), n - 1
  double* inv_w[3] = {nullptr, nullptr, nullptr};   // 1 / w_i, n
  double* wid[3] = {nullptr, nullptr, nullptr};     // w_i, n (volume weights of the gauge)
  double inv_volsum = 0.0;                          // 1 / (domain volume)
  double* host = nullptr;                           // pinned scratch (dots, coefficients)
  int device = 0;
  DevAlloc alloc;                                   // allocator of inv_dc, inv_w, wid
  ~helm_pmat() {
    for (int d = 0; d < 3; ++d)
      if (vel[d]) helm_destroy(vel[d]);
    if (pres) helm_destroy(pres);  // synchronizes the device: the vectors below are idle
    for (int d = 0; d < 3; ++d) {
      const size_t b = static_cast<size_t>(n[d]) * sizeof(double);
      alloc.put(inv_dc[d], b);
      alloc.put(inv_w[d], b);
      alloc.put(wid[d], b);
    }
    if (host) (void)hipHostFree(host);
  }
};

namespace {
constexpr int kMaxRestart = 200;

// Workspace layout for restart length m (all 256-byte aligned):
//   g[3], vsol[3]: velocity right-hand sides and solutions; vel_ws, pres_ws: solve workspaces;
//   V: (m+1) * np; Z: m * np; w, r: np; partial: (m+1) * kDotBlocks; dots: m+1; coef: m+1.
struct PmLayout {
  size_t g[3], vs[3], velws, presws, V, Z, w, r, partial, dots, coef, total;
};
PmLayout pm_layout(const helm_pmat* pm, int m) {
  PmLayout L{};
  size_t t = 0;
  for (int d = 0; d < 3; ++d) {
    L.g[d] = t;
    t += align256(pm->nv[d] * 8);
    L.vs[d] = t;
    t += align256(pm->nv[d] * 8);
  }
  L.velws = t;
  t += align256(pm->vel_ws);
  L.presws = t;
  t += align256(pm->pres_ws);
  L.V = t;
  t += align256(static_cast<size_t>(m + 1) * pm->np * 8);
  L.Z = t;
  t += align256(static_cast<size_t>(m) * pm->np * 8);
  L.w = t;
  t += align256(pm->np * 8);
  L.r = t;
  t += align256(pm->np * 8);
  L.partial = t;
  t += align256(static_cast<size_t>(m + 1) * kDotBlocks * 8);
  L.dots = t;
  t += align256(static_cast<size_t>(m + 1) * 8);
  L.coef = t;
  t += align256(static_cast<size_t>(m + 1) * 8);
  L.total = t;
  return L;
}

// y = C p
helm_status pm_apply(helm_pmat* pm, const double* p, double* y, unsigned char* ws, const PmLayout& L,
                     hipStream_t st) {
  hipError_t e = fill(y, pm->np, 0.0, st);
  for (int d = 0; d < 3 && e == hipSuccess; ++d) {
    double* g = reinterpret_cast<double*>(ws + L.g[d]);
    double* v = reinterpret_cast<double*>(ws + L.vs[d]);
    e = mac_grad(d, p, g, pm->n, pm->inv_dc[d], st);
    if (e != hipSuccess) break;
    helm_info info;
    const helm_status s = helm_solve(pm->vel[d], g, v, 1, nullptr, ws + L.velws, st, &info);
    if (s != HELM_OK) return s;
    e = mac_div_acc(d, v, y, pm->n, pm->inv_w[d], -1.0, st);
  }
  return st_from(e);
}

// host <- dot products of V[0..k) with w
helm_status dots(helm_pmat* pm, const double* V, int k, const double* w, unsigned char* ws, const PmLayout& L,
                 hipStream_t st, double* out) {
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* dd = reinterpret_cast<double*>(ws + L.dots);
  hipError_t e = multi_dot(V, pm->np, k, w, pm->np, partial, dd, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pm->host, dd, k * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = helm::wait_stream(st);
  if (e != hipSuccess) return st_from(e);
  std::memcpy(out, pm->host, k * sizeof(double));
  return HELM_OK;
}

// w += sum_j c[j] V_j  with c given on the host
helm_status axpys(helm_pmat* pm, double* w, const double* V, int k, const double* c, unsigned char* ws,
                  const PmLayout& L, hipStream_t st) {
  double* coef = reinterpret_cast<double*>(ws + L.coef);
  // the pinned buffer is reused after the copy completes (synchronous below)
  std::memcpy(pm->host, c, k * sizeof(double));
  hipError_t e = hipMemcpyAsync(coef, pm->host, k * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = multi_axpy(w, V, pm->np, k, coef, pm->np, st);
  if (e == hipSuccess) e = helm::wait_stream(st);
  return st_from(e);
}

// w += sum_j c[j] V_j (c on the host), then host <- V_j . w (j < k) and |w|^2 of the updated w,
// in one sweep; false (nothing done) when the fused kernel does not apply (k or alignment)
bool axpy_dots(helm_pmat* pm, double* w, const double* V, int k, const double* c, unsigned char* ws,
               const PmLayout& L, hipStream_t st, double* out, helm_status* s) {
  double* coef = reinterpret_cast<double*>(ws + L.coef);
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* dd = reinterpret_cast<double*>(ws + L.dots);
  if (k > kAxpyDotMax || pm->np % 2 || reinterpret_cast<uintptr_t>(V) % 16 || reinterpret_cast<uintptr_t>(w) % 16)
    return false;
  std::memcpy(pm->host, c, k * sizeof(double));
  hipError_t e = hipMemcpyAsync(coef, pm->host, k * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = multi_axpy_dot(w, V, pm->np, k, coef, pm->np, partial, dd, st);
  // the download reuses the pinned buffer after the upload (same stream, in order)
  if (e == hipSuccess) e = hipMemcpyAsync(pm->host, dd, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = helm::wait_stream(st);
  *s = st_from(e);
  if (e == hipSuccess) std::memcpy(out, pm->host, (k + 1) * sizeof(double));
  return true;
}

helm_status norm2(helm_pmat* pm, const double* x, unsigned char* ws, const PmLayout& L, hipStream_t st,
                  double* out) {
  double v = 0.0;
  const helm_status s = dots(pm, x, 1, x, ws, L, st, &v);
  *out = std::sqrt(std::max(v, 0.0));
  return s;
}
}  // namespace

extern "C" helm_status helm_pmatrix_setup(const helm_grid* p_grid, double tau, const helm_opts* opts,
                                          helm_pmat** out) {
  if (!p_grid || !out || !(tau > 0.0) || !std::isfinite(tau)) return HELM_EINVAL;
  *out = nullptr;
  std::unique_ptr<helm_pmat> pm(new (std::nothrow) helm_pmat());
  if (!pm) return HELM_ENOMEM;
  pm->tau = tau;
  if (hipGetDevice(&pm->device) != hipSuccess) return HELM_EDEVICE;
  for (int d = 0; d < 3; ++d) {
    if (!p_grid->faces[d] || p_grid->n[d] < 3) return HELM_EINVAL;
    pm->n[d] = p_grid->n[d];
  }
  pm->np = static_cast<long long>(pm->n[0]) * pm->n[1] * pm->n[2];
  // velocity plans: face-located along d, no-slip walls, sigma = 1/tau
  helm_opts vo;
  helm_default_opts(&vo);
  if (opts) vo = *opts;
  pm->alloc = DevAlloc::from(vo);
  if (!pm->alloc.valid()) return HELM_EINVAL;
  if (vo.precision != HELM_FP64) vo.method = HELM_TPF;  // the Thomas variant runs in FP64 only
  for (int d = 0; d < 3; ++d) {
    helm_grid g = *p_grid;
    for (int e = 0; e < 3; ++e) g.loc[e] = (e == d) ? HELM_FACE : HELM_CELL;
    helm_bc bc;
    for (int e = 0; e < 3; ++e) bc.lo[e] = bc.hi[e] = HELM_DIRICHLET;
    helm_status s = helm_setup(&g, &bc, 1.0 / tau, &vo, &pm->vel[d]);
    if (s != HELM_OK) return s;
    size_t b = 0;
    if ((s = helm_workspace_size(pm->vel[d], 1, &b)) != HELM_OK) return s;
    pm->vel_ws = std::max(pm->vel_ws, b);
    pm->nv[d] = pm->np / pm->n[d] * (pm->n[d] - 1);
  }
  helm_status s = helm_pressure_setup(p_grid, &vo, &pm->pres);
  if (s != HELM_OK) return s;
  if ((s = helm_workspace_size(pm->pres, 1, &pm->pres_ws)) != HELM_OK) return s;
  double volsum = 1.0;
  for (int d = 0; d < 3; ++d) {
    const int n = pm->n[d];
    const double* f = p_grid->faces[d];
    std::vector<double> idc(n - 1), iw(n), wd(n);
    double len = 0.0;
    for (int i = 0; i < n; ++i) {
      wd[i] = f[i + 1] - f[i];
      iw[i] = 1.0 / wd[i];
      len += wd[i];
    }
    volsum *= len;
    for (int i = 0; i + 1 < n; ++i) idc[i] = 1.0 / (0.5 * (f[i + 2] - f[i]));  // c_{i+1} - c_i
    // n doubles each (n - 1 used for inv_dc), so that each block is released with its size
    const size_t nb = static_cast<size_t>(n) * sizeof(double);
    hipError_t e = pm->alloc.get(reinterpret_cast<void**>(&pm->inv_dc[d]), nb);
    if (e == hipSuccess) e = pm->alloc.get(reinterpret_cast<void**>(&pm->inv_w[d]), nb);
    if (e == hipSuccess) e = pm->alloc.get(reinterpret_cast<void**>(&pm->wid[d]), nb);
    if (e == hipSuccess) e = hipMemcpy(pm->inv_dc[d], idc.data(), (n - 1) * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pm->inv_w[d], iw.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pm->wid[d], wd.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return st_from(e);
  }
  pm->inv_volsum = 1.0 / volsum;
  if (hipHostMalloc(reinterpret_cast<void**>(&pm->host), (kMaxRestart + 2) * sizeof(double)) != hipSuccess)
    return HELM_ENOMEM;
  *out = pm.release();
  return HELM_OK;
}

extern "C" helm_status helm_pmatrix_workspace_size(const helm_pmat* pm, int restart, size_t* bytes) {
  if (!pm || !bytes || restart < 1 || restart > kMaxRestart) return HELM_EINVAL;
  *bytes = pm_layout(pm, restart).total;
  return HELM_OK;
}

extern "C" helm_status helm_pmatrix_apply(helm_pmat* pm, const double* p, double* y, void* ws, void* stream) {
  if (!pm || !p || !y || !ws || p == y || reinterpret_cast<uintptr_t>(ws) % 256) return HELM_EINVAL;
  const PmLayout L = pm_layout(pm, 1);
  return pm_apply(pm, p, y, static_cast<unsigned char*>(ws), L, static_cast<hipStream_t>(stream));
}

extern "C" helm_status helm_pmatrix_solve(helm_pmat* pm, const double* b, double* p, double tol, int max_it,
                                          int restart, int use_precond, void* wsv, void* stream,
                                          helm_info* info) {
  if (!pm || !b || !p || !wsv || b == p || !(tol > 0.0) || max_it < 1 || restart < 1 || restart > kMaxRestart)
    return HELM_EINVAL;
  if (use_precond < 0 || use_precond > 2) return HELM_EINVAL;
  if (reinterpret_cast<uintptr_t>(wsv) % 256) return HELM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* ws = static_cast<unsigned char*>(wsv);
  const int m = restart;
  const PmLayout L = pm_layout(pm, m);
  const long long np = pm->np;
  double* V = reinterpret_cast<double*>(ws + L.V);
  double* Z = reinterpret_cast<double*>(ws + L.Z);
  double* w = reinterpret_cast<double*>(ws + L.w);
  double* r = reinterpret_cast<double*>(ws + L.r);
  helm_status s = HELM_OK;
  hipError_t e = fill(p, np, 0.0, st);
  if (e != hipSuccess) return st_from(e);
  double bnorm = 0.0;
  if ((s = norm2(pm, b, ws, L, st, &bnorm)) != HELM_OK) return s;
  if (info) {
    info->iterations = 0;
    info->residual = 0.0;
    info->sweeps = 0;
    info->converged = 1;
    info->last_correction = 0.0;
  }
  if (bnorm == 0.0) return HELM_OK;
  int it = 0;
  int nsolves = 0;  // Helmholtz solves: three per action of C, one per preconditioner application
  double relres = 1.0;
  std::vector<double> H(static_cast<size_t>(m + 1) * m), cs(m), sn(m), gvec(m + 1), h(m + 1), h2(m + 1);
  bool first = true;
  while (it < max_it) {
    // r = b - C p  (p = 0 on the first cycle)
    if (first) {
      e = scale(r, b, 1.0, np, st);
    } else {
      if ((s = pm_apply(pm, p, w, ws, L, st)) != HELM_OK) return s;
      nsolves += 3;
      e = scale(r, b, 1.0, np, st);
      if (e == hipSuccess) {
        const double minus1 = -1.0;
        if ((s = axpys(pm, r, w, 1, &minus1, ws, L, st)) != HELM_OK) return s;
      }
    }
    if (e != hipSuccess) return st_from(e);
    first = false;
    double beta = 0.0;
    if ((s = norm2(pm, r, ws, L, st, &beta)) != HELM_OK) return s;
    relres = beta / bnorm;
    if (relres <= tol) break;
    if ((e = scale(V, r, 1.0 / beta, np, st)) != hipSuccess) return st_from(e);
    std::fill(gvec.begin(), gvec.end(), 0.0);
    gvec[0] = beta;
    int j = 0;
    for (; j < m && it < max_it; ++j, ++it) {
      double* vj = V + j * np;
      double* zj = Z + j * np;
      // z_j = M^{-1} v_j, w = C z_j
      if (use_precond == 1 || use_precond == 2) {
        helm_info pi;
        s = helm_pressure_solve(pm->pres, vj, zj, 1, ws + L.presws, st, &pi);
        ++nsolves;
        if (s != HELM_OK && s != HELM_ENOTCONVERGED) return s;
        if (use_precond == 2) {  // z = v + sigma_v * A_p^{-1} v
          if ((e = axpby(zj, 1.0 / pm->tau, vj, 1.0, np, st)) != hipSuccess) return st_from(e);
        }
      } else {
        if ((e = scale(zj, vj, 1.0, np, st)) != hipSuccess) return st_from(e);
      }
      // w = C z_j is built in the basis slot j + 1, so that one multi-dot over V_0 .. V_{j+1}
      // gives the projections and |w|^2 together
      double* wv = V + (j + 1) * np;
      if ((s = pm_apply(pm, zj, wv, ws, L, st)) != HELM_OK) return s;
      nsolves += 3;
      // classical Gram-Schmidt with selective reorthogonalization (Daniel, Gragg, Kaufman &
      // Stewart 1976): the norm after a pass follows from Pythagoras, |w'|^2 = |w|^2 - |h|^2;
      // a second pass runs only when that cancels more than half of |w|^2 (eta = 1/sqrt 2),
      // and an explicit norm only if the second pass cancels too
      std::fill(h.begin(), h.end(), 0.0);
      double hn = -1.0;
      // With the fused sweep, the first pass's update and the second pass's projections (and
      // the exact |w'|^2) share one sweep over V; the second update runs only if needed.
      bool fused = false;
      {
        if ((s = dots(pm, V, j + 2, wv, ws, L, st, h2.data())) != HELM_OK) return s;
        const double ww = h2[j + 1];
        std::vector<double> c(j + 1), d2(j + 2);
        for (int i = 0; i <= j; ++i) {
          h[i] = h2[i];
          c[i] = -h2[i];
        }
        helm_status sf = HELM_OK;
        fused = axpy_dots(pm, wv, V, j + 1, c.data(), ws, L, st, d2.data(), &sf);
        if (sf != HELM_OK) return sf;
        if (fused) {
          const double ww2 = d2[j + 1];
          if (ww2 > 0.5 * ww) {
            hn = std::sqrt(ww2);  // little cancellation: the remaining projections are dropped
          } else {
            double hh = 0.0;
            for (int i = 0; i <= j; ++i) {
              h[i] += d2[i];
              c[i] = -d2[i];
              hh += d2[i] * d2[i];
            }
            if ((s = axpys(pm, wv, V, j + 1, c.data(), ws, L, st)) != HELM_OK) return s;
            const double est = ww2 - hh;
            if (est > 0.5 * ww2) hn = std::sqrt(est);
          }
        } else {
          // separate passes: finish the first one here
          double hh = 0.0;
          for (int i = 0; i <= j; ++i) hh += h2[i] * h2[i];
          if ((s = axpys(pm, wv, V, j + 1, c.data(), ws, L, st)) != HELM_OK) return s;
          const double est = ww - hh;
          if (est > 0.5 * ww) hn = std::sqrt(est);
        }
      }
      for (int pass = 1; pass < 2 && hn < 0.0 && !fused; ++pass) {
        if ((s = dots(pm, V, j + 2, wv, ws, L, st, h2.data())) != HELM_OK) return s;
        const double ww = h2[j + 1];
        double hh = 0.0;
        std::vector<double> c(j + 1);
        for (int i = 0; i <= j; ++i) {
          h[i] += h2[i];
          c[i] = -h2[i];
          hh += h2[i] * h2[i];
        }
        if ((s = axpys(pm, wv, V, j + 1, c.data(), ws, L, st)) != HELM_OK) return s;
        const double est = ww - hh;
        if (est > 0.5 * ww) hn = std::sqrt(est);
      }
      if (hn < 0.0 && (s = norm2(pm, wv, ws, L, st, &hn)) != HELM_OK) return s;
      h[j + 1] = hn;
      if (hn > 0.0) {
        if ((e = scale(wv, wv, 1.0 / hn, np, st)) != hipSuccess) return st_from(e);
      }
      // apply previous rotations, then a new one to annihilate h[j+1]
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double rr = std::hypot(h[j], h[j + 1]);
      cs[j] = rr > 0.0 ? h[j] / rr : 1.0;
      sn[j] = rr > 0.0 ? h[j + 1] / rr : 0.0;
      h[j] = rr;
      h[j + 1] = 0.0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = cs[j] * gvec[j];
      for (int i = 0; i <= j; ++i) H[static_cast<size_t>(i) * m + j] = h[i];
      relres = std::fabs(gvec[j + 1]) / bnorm;
      if (relres <= tol || hn == 0.0) {
        ++j;
        ++it;
        break;
      }
    }
    // y = R^{-1} g, p += Z y
    std::vector<double> y(j);
    for (int i = j - 1; i >= 0; --i) {
      double t = gvec[i];
      for (int k = i + 1; k < j; ++k) t -= H[static_cast<size_t>(i) * m + k] * y[k];
      y[i] = t / H[static_cast<size_t>(i) * m + i];
    }
    if (j > 0 && (s = axpys(pm, p, Z, j, y.data(), ws, L, st)) != HELM_OK) return s;
    if (relres <= tol) {
      // confirm with the true residual
      if ((s = pm_apply(pm, p, w, ws, L, st)) != HELM_OK) return s;
      nsolves += 3;
      if ((e = scale(r, b, 1.0, np, st)) != hipSuccess) return st_from(e);
      const double minus1 = -1.0;
      if ((s = axpys(pm, r, w, 1, &minus1, ws, L, st)) != HELM_OK) return s;
      double rn = 0.0;
      if ((s = norm2(pm, r, ws, L, st, &rn)) != HELM_OK) return s;
      relres = rn / bnorm;
      if (relres <= tol) break;
    }
  }
  if (info) {
    info->iterations = it;
    info->residual = relres;
    info->converged = relres <= tol;
    info->sweeps = nsolves;
  }
  return relres <= tol ? HELM_OK : HELM_ENOTCONVERGED;
}

// ---- Stokes system (Section 2, eq. 8) by the three-step factorization ----
// With the momentum rows in the library's sign (H_d u_d + Grad_d p = f_d, sum_d Div_d u_d = g):
//   1. u^_d = H_d^{-1} f_d                       (three velocity solves)
//   2. C p = g - sum_d Div_d u^_d                 (FGMRES on the pressure matrix)
//   3. u_d = u^_d - H_d^{-1} Grad_d p             (three more velocity solves)
// The velocities vanish on the walls, so Div u^ has zero volume-weighted mean and the
// right-hand side of step 2 is compatible once that mean is removed from g.
namespace {
struct StokesLayout {
  PmLayout pm;
  size_t b, mean, total;
};
StokesLayout stokes_layout(const helm_pmat* pm, int m) {
  StokesLayout L{};
  L.pm = pm_layout(pm, m);
  size_t t = L.pm.total;
  L.b = t;
  t += align256(pm->np * 8);
  L.mean = t;
  t += align256((kMeanBlocks + 1) * 8);
  L.total = t;
  return L;
}
}  // namespace

extern "C" helm_status helm_stokes_workspace_size(const helm_pmat* pm, int restart, size_t* bytes) {
  if (!pm || !bytes || restart < 1 || restart > kMaxRestart) return HELM_EINVAL;
  *bytes = stokes_layout(pm, restart).total;
  return HELM_OK;
}

extern "C" helm_status helm_stokes_solve(helm_pmat* pm, const double* const f[3], const double* g,
                                         double* const u[3], double* p, double tol, int max_it, int restart,
                                         int use_precond, void* wsv, void* stream, helm_info* info) {
  if (!pm || !f || !u || !p || !wsv || !(tol > 0.0) || max_it < 1 || restart < 1 || restart > kMaxRestart)
    return HELM_EINVAL;
  if (use_precond < 0 || use_precond > 2 || reinterpret_cast<uintptr_t>(wsv) % 256) return HELM_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!f[d] || !u[d] || f[d] == u[d] || u[d] == p || static_cast<const double*>(u[d]) == g) return HELM_EINVAL;
    for (int e = 0; e < d; ++e)
      if (u[e] == u[d]) return HELM_EINVAL;
  }
  if (g == p) return HELM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* ws = static_cast<unsigned char*>(wsv);
  const StokesLayout L = stokes_layout(pm, restart);
  double* b = reinterpret_cast<double*>(ws + L.b);
  helm_status s = HELM_OK;
  // 1. u^ = H^{-1} f, held in u
  for (int d = 0; d < 3 && s == HELM_OK; ++d) {
    helm_info vi;
    s = helm_solve(pm->vel[d], f[d], u[d], 1, nullptr, ws + L.pm.velws, st, &vi);
  }
  if (s != HELM_OK) return s;
  // 2. b = P_V (g - sum Div u^), then C p = b
  hipError_t e = g ? scale(b, g, 1.0, pm->np, st) : fill(b, pm->np, 0.0, st);
  for (int d = 0; d < 3 && e == hipSuccess; ++d) e = mac_div_acc(d, u[d], b, pm->n, pm->inv_w[d], -1.0, st);
  if (e == hipSuccess)
    e = remove_mean(b, pm->wid[0], pm->wid[1], pm->wid[2], pm->n[0], pm->n[1], pm->n[2], 1, pm->inv_volsum, 1ull,
                    reinterpret_cast<double*>(ws + L.mean), st);
  if (e != hipSuccess) return st_from(e);
  helm_info ci;
  const helm_status sc = helm_pmatrix_solve(pm, b, p, tol, max_it, restart, use_precond, wsv, stream, &ci);
  if (sc != HELM_OK && sc != HELM_ENOTCONVERGED) return sc;
  // 3. u -= H^{-1} Grad p
  for (int d = 0; d < 3 && s == HELM_OK; ++d) {
    double* gv = reinterpret_cast<double*>(ws + L.pm.g[d]);
    double* t = reinterpret_cast<double*>(ws + L.pm.vs[d]);
    if ((e = mac_grad(d, p, gv, pm->n, pm->inv_dc[d], st)) != hipSuccess) return st_from(e);
    helm_info vi;
    s = helm_solve(pm->vel[d], gv, t, 1, nullptr, ws + L.pm.velws, st, &vi);
    if (s == HELM_OK && (e = axpby(u[d], 1.0, t, -1.0, pm->nv[d], st)) != hipSuccess) return st_from(e);
  }
  if (s != HELM_OK) return s;
  if (info) {
    info->iterations = ci.iterations;
    info->residual = ci.residual;
    info->converged = ci.converged;
    info->sweeps = 6 + ci.sweeps;
    info->last_correction = 0.0;
  }
  return sc;
}

extern "C" void helm_pmatrix_destroy(helm_pmat* pm) {
  if (!pm) return;
  (void)hipDeviceSynchronize();
  delete pm;
}
