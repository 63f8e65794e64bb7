// One step of the paper's time integration (Section 5, eqs. 37-40): Boussinesq convection in a
// box on the MAC grid, second-order backward differences in time, incremental pressure
// correction.  Per step: right-hand sides formed from the previous fields (time derivative
// terms, conservative central advection, pressure gradient, buoyancy, the heated-wall values),
// one temperature and three velocity Helmholtz solves, one pressure Poisson solve, the velocity
// correction and the pressure update.  The solves go to plans of the stepper or, when a server
// is given, to that server as requests (the temperature first, then the three velocities
// together, then the pressure), so the step drives the serving path with the solve mix of a
// time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <vector>

#include "../../include/helm.h"
#include "alloc.hpp"
#include "kernels.hpp"

namespace helm {
namespace {

struct TsGeom {
  int n[3];             // pressure cells per axis
  const double* w[3];   // cell widths
  const double* idc[3]; // 1 / (c_{i+1} - c_i), n - 1 entries
  const double* iw[3];  // 1 / w_i
};

// Velocity component d on the face grid of d (n[d] - 1 interior faces along d), at coordinates
// c with c[d] the face index m in 0..n[d] (the two wall faces carry 0).
__device__ inline double vel_at(const double* __restrict__ v, int d, const TsGeom& g, int c0, int c1, int c2) {
  int c[3] = {c0, c1, c2};
  const int m = c[d];
  if (m <= 0 || m >= g.n[d]) return 0.0;
  c[d] = m - 1;
  int nv[3] = {g.n[0], g.n[1], g.n[2]};
  nv[d] -= 1;
  return v[(static_cast<long long>(c[2]) * nv[1] + c[1]) * nv[0] + c[0]];
}

__device__ inline double cell_at(const double* __restrict__ a, const TsGeom& g, int i, int j, int k) {
  return a[(static_cast<long long>(k) * g.n[1] + j) * g.n[0] + i];
}

// (37): f_T = ((4 T0 - Tm) / (2 dt) - A_T(v0, T0) + kappa * wall) / kappa at every cell.
__global__ __launch_bounds__(256) void k_ts_rhs_T(const double* __restrict__ T0, const double* __restrict__ Tm,
                                                  const double* __restrict__ vx, const double* __restrict__ vy,
                                                  const double* __restrict__ vz, double* __restrict__ out, TsGeom g,
                                                  double dt, double kappa, double wall_lo, double wall_hi) {
  const long long P = static_cast<long long>(g.n[0]) * g.n[1] * g.n[2];
  const double* v[3] = {vx, vy, vz};
  for (long long id = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; id < P;
       id += static_cast<long long>(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(id % g.n[0]);
    const int j = static_cast<int>((id / g.n[0]) % g.n[1]);
    const int k = static_cast<int>(id / (static_cast<long long>(g.n[0]) * g.n[1]));
    const int c[3] = {i, j, k};
    double adv = 0.0;
    for (int d = 0; d < 3; ++d) {
      // fluxes through the cell's lower and upper d-faces: V * (mean of the two cells)
      double F[2];
      for (int s = 0; s < 2; ++s) {
        const int m = c[d] + s;  // face index
        int lo[3] = {i, j, k}, hi[3] = {i, j, k}, at[3] = {i, j, k};
        lo[d] = max(m - 1, 0);
        hi[d] = min(m, g.n[d] - 1);
        at[d] = m;
        const double V = vel_at(v[d], d, g, at[0], at[1], at[2]);
        F[s] = V * 0.5 * (cell_at(T0, g, lo[0], lo[1], lo[2]) + cell_at(T0, g, hi[0], hi[1], hi[2]));
      }
      adv += (F[1] - F[0]) * g.iw[d][c[d]];
    }
    double wall = 0.0;
    if (i == 0) wall += wall_lo;
    if (i == g.n[0] - 1) wall += wall_hi;
    out[id] = ((4.0 * T0[id] - Tm[id]) / (2.0 * dt) - adv + kappa * wall) / kappa;
  }
}

// (38): f_d = ((4 v0_d - vm_d) / (2 dt) - A_d(v0) - Grad_d p0 + [d = z] T1 at the face) / nu on
// the d-face grid.
template <int D>
__global__ __launch_bounds__(256) void k_ts_rhs_vel(const double* __restrict__ vx, const double* __restrict__ vy,
                                                    const double* __restrict__ vz, const double* __restrict__ vm,
                                                    const double* __restrict__ p0, const double* __restrict__ T1,
                                                    double* __restrict__ out, TsGeom g, double dt, double nu) {
  int nv[3] = {g.n[0], g.n[1], g.n[2]};
  nv[D] -= 1;
  const long long P = static_cast<long long>(nv[0]) * nv[1] * nv[2];
  const double* v[3] = {vx, vy, vz};
  const double* ud = v[D];
  for (long long id = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; id < P;
       id += static_cast<long long>(gridDim.x) * blockDim.x) {
    int c[3];
    c[0] = static_cast<int>(id % nv[0]);
    c[1] = static_cast<int>((id / nv[0]) % nv[1]);
    c[2] = static_cast<int>(id / (static_cast<long long>(nv[0]) * nv[1]));
    const int f = c[D];  // the point sits on face f + 1, between cells f and f + 1 along D
    // along D: flux ubar^2 at the two cell centres beside the face
    auto U = [&](int m) {  // v_D on face m of the same row
      int a[3] = {c[0], c[1], c[2]};
      a[D] = m;
      return vel_at(ud, D, g, a[0], a[1], a[2]);
    };
    const double ub0 = 0.5 * (U(f) + U(f + 1)), ub1 = 0.5 * (U(f + 1) + U(f + 2));
    double adv = (ub1 * ub1 - ub0 * ub0) * g.idc[D][f];
    for (int e = 0; e < 3; ++e) {
      if (e == D) continue;
      const int ce = c[e];
      double G[2];
      for (int s = 0; s < 2; ++s) {
        const int m = ce + s;  // e-face index
        // v_e on this e-face in the two cells beside the D-face (zero on e-walls)
        int a[3] = {c[0], c[1], c[2]};
        a[e] = m;
        a[D] = f;
        const double ve0 = vel_at(v[e], e, g, a[0], a[1], a[2]);
        a[D] = f + 1;
        const double ve1 = vel_at(v[e], e, g, a[0], a[1], a[2]);
        // v_D in the two e-neighbours of the e-face (clamped at the walls, where the flux is 0)
        int b0[3] = {c[0], c[1], c[2]}, b1[3] = {c[0], c[1], c[2]};
        b0[e] = max(m - 1, 0);
        b1[e] = min(m, g.n[e] - 1);
        const double u0 = ud[(static_cast<long long>(b0[2]) * nv[1] + b0[1]) * nv[0] + b0[0]];
        const double u1 = ud[(static_cast<long long>(b1[2]) * nv[1] + b1[1]) * nv[0] + b1[0]];
        G[s] = 0.5 * (ve0 + ve1) * 0.5 * (u0 + u1);
      }
      adv += (G[1] - G[0]) * g.iw[e][ce];
    }
    int lo[3] = {c[0], c[1], c[2]}, hi[3] = {c[0], c[1], c[2]};
    hi[D] = f + 1;
    const double grad =
        (cell_at(p0, g, hi[0], hi[1], hi[2]) - cell_at(p0, g, lo[0], lo[1], lo[2])) * g.idc[D][f];
    double rhs = (4.0 * ud[id] - vm[id]) / (2.0 * dt) - adv - grad;
    if constexpr (D == 2) rhs += 0.5 * (cell_at(T1, g, lo[0], lo[1], lo[2]) + cell_at(T1, g, hi[0], hi[1], hi[2]));
    out[id] = rhs / nu;
  }
}

dim3 grid_for(long long n) { return dim3(static_cast<unsigned>(std::min<long long>((n + 255) / 256, 8192))); }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

helm_status st_from(hipError_t e) {
  if (e == hipSuccess) return HELM_OK;
  return e == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EDEVICE;
}

}  // namespace
}  // namespace helm

using namespace helm;

struct helm_ts {
  int n[3] = {0, 0, 0};
  double Pr = 0, Gr = 0, dt = 0, T_lo = 0, T_hi = 0;
  double kappa = 0, nu = 0, sig_T = 0, sig_v = 0, wall_lo = 0, wall_hi = 0;
  std::vector<double> faces[3];
  helm_plan* planT = nullptr;
  helm_plan* planV[3] = {nullptr, nullptr, nullptr};
  helm_plan* planP = nullptr;
  size_t solve_ws = 0;
  long long Pc = 0, Pv[3] = {0, 0, 0};
  DevAlloc alloc;
  double* geo = nullptr;  // w, 1/dc, 1/w per axis, on the device
  size_t geo_bytes = 0;
  TsGeom g{};
  long long next_id = 0;
  ~helm_ts() {
    if (planT) helm_destroy(planT);  // synchronizes the device
    for (auto* p : planV)
      if (p) helm_destroy(p);
    if (planP) helm_destroy(planP);
    alloc.put(geo, geo_bytes);
  }
};

namespace {
// workspace: f_T | f_v[3] | div | dp | grad scratch | solve workspace
struct TsLayout {
  size_t fT, fv[3], div, dp, tmp, solve, total;
};
TsLayout ts_layout(const helm_ts* ts) {
  TsLayout L{};
  size_t t = 0;
  L.fT = t;
  t += align256(ts->Pc * 8);
  long long vmax = 0;
  for (int d = 0; d < 3; ++d) {
    L.fv[d] = t;
    t += align256(ts->Pv[d] * 8);
    vmax = std::max(vmax, ts->Pv[d]);
  }
  L.div = t;
  t += align256(ts->Pc * 8);
  L.dp = t;
  t += align256(ts->Pc * 8);
  L.tmp = t;
  t += align256(vmax * 8);
  L.solve = t;
  t += align256(ts->solve_ws);
  L.total = t;
  return L;
}
}  // namespace

extern "C" helm_status helm_ts_create(const helm_grid* grid, double Pr, double Gr, double dt, double T_lo, double T_hi,
                                      const helm_opts* opts, helm_ts** out) {
  if (!grid || !out || !(Pr > 0) || !(Gr > 0) || !(dt > 0) || !std::isfinite(T_lo) || !std::isfinite(T_hi))
    return HELM_EINVAL;
  *out = nullptr;
  std::unique_ptr<helm_ts> ts(new (std::nothrow) helm_ts());
  if (!ts) return HELM_ENOMEM;
  helm_opts o;
  helm_default_opts(&o);
  if (opts) o = *opts;
  ts->alloc = DevAlloc::from(o);
  if (!ts->alloc.valid()) return HELM_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (!grid->faces[d] || grid->n[d] < 3) return HELM_EINVAL;
    ts->n[d] = grid->n[d];
    ts->faces[d].assign(grid->faces[d], grid->faces[d] + grid->n[d] + 1);
    for (int i = 0; i < grid->n[d]; ++i)
      if (!(ts->faces[d][i + 1] > ts->faces[d][i])) return HELM_EINVAL;
  }
  ts->Pr = Pr;
  ts->Gr = Gr;
  ts->dt = dt;
  ts->T_lo = T_lo;
  ts->T_hi = T_hi;
  ts->kappa = 1.0 / (Pr * std::sqrt(Gr));
  ts->nu = 1.0 / std::sqrt(Gr);
  ts->sig_T = 1.5 / (dt * ts->kappa);
  ts->sig_v = 1.5 / (dt * ts->nu);
  // wall values of T enter the cells next to the heated walls through the boundary flux
  const std::vector<double>& fx = ts->faces[0];
  const int nx = ts->n[0];
  ts->wall_lo = T_lo / ((0.5 * (fx[0] + fx[1]) - fx[0]) * (fx[1] - fx[0]));
  ts->wall_hi = T_hi / ((fx[nx] - 0.5 * (fx[nx - 1] + fx[nx])) * (fx[nx] - fx[nx - 1]));
  ts->Pc = static_cast<long long>(ts->n[0]) * ts->n[1] * ts->n[2];
  helm_grid g = *grid;
  for (int d = 0; d < 3; ++d) g.loc[d] = HELM_CELL;
  helm_bc bcT;
  for (int d = 0; d < 3; ++d) bcT.lo[d] = bcT.hi[d] = (d == 0) ? HELM_DIRICHLET : HELM_NEUMANN;
  helm_status s = helm_setup(&g, &bcT, ts->sig_T, &o, &ts->planT);
  if (s != HELM_OK) return s;
  size_t b = 0;
  if ((s = helm_workspace_size(ts->planT, 1, &b)) != HELM_OK) return s;
  ts->solve_ws = b;
  for (int d = 0; d < 3; ++d) {
    helm_grid gv = g;
    gv.loc[d] = HELM_FACE;
    helm_bc bcv;
    for (int e = 0; e < 3; ++e) bcv.lo[e] = bcv.hi[e] = HELM_DIRICHLET;
    if ((s = helm_setup(&gv, &bcv, ts->sig_v, &o, &ts->planV[d])) != HELM_OK) return s;
    if ((s = helm_workspace_size(ts->planV[d], 1, &b)) != HELM_OK) return s;
    ts->solve_ws = std::max(ts->solve_ws, b);
    ts->Pv[d] = ts->Pc / ts->n[d] * (ts->n[d] - 1);
  }
  if ((s = helm_pressure_setup(&g, &o, &ts->planP)) != HELM_OK) return s;
  if ((s = helm_workspace_size(ts->planP, 1, &b)) != HELM_OK) return s;
  ts->solve_ws = std::max(ts->solve_ws, b);
  // geometry on the device: per axis w[n], 1/dc[n-1], 1/w[n]
  std::vector<double> host;
  size_t off[3][3];
  for (int d = 0; d < 3; ++d) {
    const std::vector<double>& f = ts->faces[d];
    const int n = ts->n[d];
    off[d][0] = host.size();
    for (int i = 0; i < n; ++i) host.push_back(f[i + 1] - f[i]);
    off[d][1] = host.size();
    for (int i = 0; i + 1 < n; ++i) host.push_back(1.0 / (0.5 * (f[i + 2] - f[i])));
    off[d][2] = host.size();
    for (int i = 0; i < n; ++i) host.push_back(1.0 / (f[i + 1] - f[i]));
  }
  ts->geo_bytes = host.size() * sizeof(double);
  void* p = nullptr;
  hipError_t e = ts->alloc.get(&p, ts->geo_bytes);
  if (e != hipSuccess) return st_from(e);
  ts->geo = static_cast<double*>(p);
  if ((e = hipMemcpy(ts->geo, host.data(), ts->geo_bytes, hipMemcpyHostToDevice)) != hipSuccess) return st_from(e);
  for (int d = 0; d < 3; ++d) {
    ts->g.n[d] = ts->n[d];
    ts->g.w[d] = ts->geo + off[d][0];
    ts->g.idc[d] = ts->geo + off[d][1];
    ts->g.iw[d] = ts->geo + off[d][2];
  }
  *out = ts.release();
  return HELM_OK;
}

extern "C" helm_status helm_ts_workspace_size(const helm_ts* ts, size_t* bytes) {
  if (!ts || !bytes) return HELM_EINVAL;
  *bytes = ts_layout(ts).total;
  return HELM_OK;
}

namespace {
// Submits the given solves to the server and waits for them (the server is dedicated to the
// stepper: its completion records are consumed here).
helm_status serve(helm_ts* ts, helm_server* srv, int count, const helm_grid* grids, const helm_bc* bcs,
                  const double* sigmas, const double* const* f, double* const* u, hipStream_t st, int* sweeps) {
  for (int q = 0; q < count; ++q) {
    const helm_status s = helm_server_submit(srv, &grids[q], &bcs[q], &sigmas[q], 1, f[q], u[q], ts->next_id++, st);
    if (s != HELM_OK) return s;
  }
  helm_status s = helm_server_drain(srv);
  if (s != HELM_OK) return s;
  helm_request_record rec[8];
  int got = 0, n = 0;
  helm_status worst = HELM_OK;
  while (got < count) {
    if ((s = helm_server_poll(srv, rec, 8, &n, 1000)) != HELM_OK) return s;
    if (n == 0) return HELM_EDEVICE;
    for (int i = 0; i < n; ++i) {
      if (rec[i].status != HELM_OK && worst == HELM_OK) worst = static_cast<helm_status>(rec[i].status);
      *sweeps += rec[i].sweeps;
    }
    got += n;
  }
  return worst;
}
}  // namespace

extern "C" helm_status helm_ts_step(helm_ts* ts, const helm_ts_fields* fl, helm_server* srv, void* wsv, void* stream,
                                    helm_info* info) {
  if (!ts || !fl || !wsv || reinterpret_cast<uintptr_t>(wsv) % 256) return HELM_EINVAL;
  if (!fl->T0 || !fl->Tm || !fl->p0 || !fl->T1 || !fl->p1) return HELM_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!fl->v0[d] || !fl->vm[d] || !fl->v1[d]) return HELM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* ws = static_cast<unsigned char*>(wsv);
  const TsLayout L = ts_layout(ts);
  double* fT = reinterpret_cast<double*>(ws + L.fT);
  double* fv[3];
  for (int d = 0; d < 3; ++d) fv[d] = reinterpret_cast<double*>(ws + L.fv[d]);
  double* div = reinterpret_cast<double*>(ws + L.div);
  double* dp = reinterpret_cast<double*>(ws + L.dp);
  double* tmp = reinterpret_cast<double*>(ws + L.tmp);
  void* sws = ws + L.solve;
  const TsGeom& g = ts->g;
  int sweeps = 0;
  helm_info si{};
  helm_status s = HELM_OK;
  // cell grid, velocity grids and walls of the requests
  helm_grid gc;
  for (int d = 0; d < 3; ++d) {
    gc.n[d] = ts->n[d];
    gc.faces[d] = ts->faces[d].data();
    gc.loc[d] = HELM_CELL;
  }
  // (37)
  hipLaunchKernelGGL(k_ts_rhs_T, grid_for(ts->Pc), dim3(256), 0, st, fl->T0, fl->Tm, fl->v0[0], fl->v0[1], fl->v0[2],
                     fT, g, ts->dt, ts->kappa, ts->wall_lo, ts->wall_hi);
  if (hipGetLastError() != hipSuccess) return HELM_EDEVICE;
  if (srv) {
    helm_bc bcT;
    for (int d = 0; d < 3; ++d) bcT.lo[d] = bcT.hi[d] = (d == 0) ? HELM_DIRICHLET : HELM_NEUMANN;
    const double* f1[1] = {fT};
    double* u1[1] = {fl->T1};
    s = serve(ts, srv, 1, &gc, &bcT, &ts->sig_T, f1, u1, st, &sweeps);
  } else {
    s = helm_solve(ts->planT, fT, fl->T1, 1, nullptr, sws, st, &si);
    sweeps += si.sweeps;
  }
  if (s != HELM_OK) return s;
  // (38)
  hipLaunchKernelGGL(k_ts_rhs_vel<0>, grid_for(ts->Pv[0]), dim3(256), 0, st, fl->v0[0], fl->v0[1], fl->v0[2],
                     fl->vm[0], fl->p0, fl->T1, fv[0], g, ts->dt, ts->nu);
  hipLaunchKernelGGL(k_ts_rhs_vel<1>, grid_for(ts->Pv[1]), dim3(256), 0, st, fl->v0[0], fl->v0[1], fl->v0[2],
                     fl->vm[1], fl->p0, fl->T1, fv[1], g, ts->dt, ts->nu);
  hipLaunchKernelGGL(k_ts_rhs_vel<2>, grid_for(ts->Pv[2]), dim3(256), 0, st, fl->v0[0], fl->v0[1], fl->v0[2],
                     fl->vm[2], fl->p0, fl->T1, fv[2], g, ts->dt, ts->nu);
  if (hipGetLastError() != hipSuccess) return HELM_EDEVICE;
  if (srv) {
    helm_grid gv[3];
    helm_bc bv[3];
    double sv[3];
    const double* fs[3];
    double* us[3];
    for (int d = 0; d < 3; ++d) {
      gv[d] = gc;
      gv[d].loc[d] = HELM_FACE;
      for (int e = 0; e < 3; ++e) bv[d].lo[e] = bv[d].hi[e] = HELM_DIRICHLET;
      sv[d] = ts->sig_v;
      fs[d] = fv[d];
      us[d] = fl->v1[d];
    }
    s = serve(ts, srv, 3, gv, bv, sv, fs, us, st, &sweeps);
  } else {
    for (int d = 0; d < 3 && s == HELM_OK; ++d) {
      s = helm_solve(ts->planV[d], fv[d], fl->v1[d], 1, nullptr, sws, st, &si);
      sweeps += si.sweeps;
    }
  }
  if (s != HELM_OK) return s;
  // (39): -Lap dp = Div v* / dt
  hipError_t e = fill(div, ts->Pc, 0.0, st);
  for (int d = 0; d < 3 && e == hipSuccess; ++d) e = mac_div_acc(d, fl->v1[d], div, ts->n, g.iw[d], 1.0 / ts->dt, st);
  if (e != hipSuccess) return st_from(e);
  if (srv) {
    helm_bc bp;
    for (int d = 0; d < 3; ++d) bp.lo[d] = bp.hi[d] = HELM_NEUMANN;
    const double zero = 0.0;
    const double* f1[1] = {div};
    double* u1[1] = {dp};
    s = serve(ts, srv, 1, &gc, &bp, &zero, f1, u1, st, &sweeps);
  } else {
    s = helm_pressure_solve(ts->planP, div, dp, 1, sws, st, &si);
    sweeps += si.sweeps;
  }
  if (s != HELM_OK) return s;
  // (40): v1 = v* + dt Grad dp;  p1 = p0 - dp (the update consistent with eq. 38's -Grad p)
  for (int d = 0; d < 3 && e == hipSuccess; ++d) {
    e = mac_grad(d, dp, tmp, ts->n, g.idc[d], st);
    if (e == hipSuccess) e = axpby(fl->v1[d], 1.0, tmp, ts->dt, ts->Pv[d], st);
  }
  if (e == hipSuccess && fl->p1 != fl->p0) e = scale(fl->p1, fl->p0, 1.0, ts->Pc, st);
  if (e == hipSuccess) e = axpby(fl->p1, 1.0, dp, -1.0, ts->Pc, st);
  if (e != hipSuccess) return st_from(e);
  if (info) {
    info->sweeps = sweeps;
    info->last_correction = 0.0;
    info->converged = 1;
    info->iterations = 0;
    info->residual = 0.0;
  }
  return HELM_OK;
}

extern "C" void helm_ts_destroy(helm_ts* ts) { delete ts; }
