// Solver driver and C ABI (include/helm.h).
//
// helm_setup builds the per-axis 1D operators and eigenpairs on the host (Section 3,
// eqs. 23-24), uploads them once, and helm_solve sequences the device kernels:
//   TPF   (eq. 29):  x-fwd -> y-fwd -> z-fwd + divide (eqs. 26-28) -> z-inv -> y-inv -> x-inv
//   TPT_Z         :  x-fwd -> y-fwd -> Thomas along z -> y-inv -> x-inv
// In the low-precision forms the products run in FP32 or BF16 and the result is refined:
//   u = M^{-1} f;  repeat r = f - H u (FP64 7-point), u += M^{-1} r  until max|du| <= tol max|u|.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <optional>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/helm.h"
#include "alloc.hpp"
#include "fft.hpp"
#include "kernels.hpp"
#include "setup.hpp"
#include "solve_impl.hpp"

using namespace helm;

namespace {

// Device blocks owned by one object, released (on its device, after a device synchronization,
// since enqueued work may still read them) through the allocator that made them.
struct DevBlocks {
  DevAlloc alloc;
  int device = 0;
  std::vector<std::pair<void*, size_t>> blocks;
  template <typename T>
  hipError_t upload(T** dst, const T* src, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void* p = nullptr;
    hipError_t e = alloc.get(&p, bytes);
    if (e != hipSuccess) return e;
    blocks.push_back({p, bytes});
    *dst = static_cast<T*>(p);
    if (count) e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    return e;
  }
  ~DevBlocks() {
    if (blocks.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    if (alloc.alloc) (void)hipDeviceSynchronize();  // a caller's allocator may reuse the block at once
    for (auto& b : blocks) alloc.put(b.first, b.second);
    (void)hipSetDevice(cur);
  }
};

// Device copy of one axis' operator and eigenbasis.  Shared between plans through a
// reference-counted cache keyed by the axis definition (faces, location, walls, device,
// allocator).
struct DevAxis {
  Axis1D host;
  std::string key;           // cache key (faces, location, walls, device, allocator)
  DevBlocks mem;             // every device buffer below
  int device = 0;
  double* lam = nullptr;     // m eigenvalues
  double* coef = nullptr;    // 3m: lower, diag, upper rows of A
  double* kdiag = nullptr;   // m   (Thomas)
  double* koff = nullptr;    // m-1 (Thomas)
  double* vol = nullptr;     // m
  double* E = nullptr;       // m*m row-major
  double* Einv = nullptr;    // m*m row-major
  double* gdiag = nullptr;   // radial axis: dr / rc (Thomas metric term)
  double* inv_r2 = nullptr;  // radial axis: 1 / rc^2 (stencil metric)
  bool fft_ok = false;       // uniform axis with a fast sine/cosine transform (HELM_FFT)
  FftTables fft[2];          // [forward (E^{-1}), inverse (E)]
  void* sw[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // [prec][fwd, inv]
  void* sw3[2] = {nullptr, nullptr};  // split-BF16 pieces [fwd, inv]
};

// How an axis' 1D operator is built: Cartesian (eq. 23), or the radial and periodic-theta
// axes of the cylindrical operator (Section 6, eq. 41).
enum AxisKind : int { AXIS_CART = 0, AXIS_RADIAL = 1, AXIS_PERIODIC = 2 };

std::string build_axis(int kind, int n, const double* faces, int loc, int lo, int hi, Axis1D& h) {
  if (kind == AXIS_RADIAL) return build_operator_radial(n, faces, lo, hi, h);
  if (kind == AXIS_PERIODIC) return build_operator_periodic(n, faces, h);
  return build_operator_1d(n, faces, loc, lo, hi, h);
}

std::mutex g_cache_mu;
std::map<std::string, std::weak_ptr<DevAxis>> g_cache;

// Drops the entries of a weak cache whose object is gone (keys hold whole face arrays).
template <typename T>
void purge_expired(std::map<std::string, std::weak_ptr<T>>& m) {
  for (auto it = m.begin(); it != m.end();) it = it->second.expired() ? m.erase(it) : std::next(it);
}

helm_status from_hip(hipError_t e) {
  if (e == hipSuccess) return HELM_OK;
  if (e == hipErrorOutOfMemory) return HELM_ENOMEM;
  return HELM_EDEVICE;
}

std::string axis_key(int kind, int n, const double* faces, int loc, int lo, int hi, int device, const DevAlloc& al) {
  std::string k(reinterpret_cast<const char*>(faces), sizeof(double) * (n + 1));
  k.push_back(static_cast<char>(kind));
  k.push_back(static_cast<char>(loc));
  k.push_back(static_cast<char>(lo));
  k.push_back(static_cast<char>(hi));
  k.append(reinterpret_cast<const char*>(&device), sizeof(int));
  k.append(al.key());
  return k;
}

// build = false: a cache lookup only (out stays empty when the axis is not resident).
helm_status get_axis(int kind, int n, const double* faces, int loc, int lo, int hi, const DevAlloc& al,
                     std::shared_ptr<DevAxis>& out, bool build = true) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HELM_EDEVICE;
  const std::string key = axis_key(kind, n, faces, loc, lo, hi, dev, al);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      out = it->second.lock();
      if (out) return HELM_OK;
    }
  }
  if (!build) return HELM_OK;
  auto ax = std::make_shared<DevAxis>();
  ax->device = dev;
  ax->key = key;
  ax->mem.alloc = al;
  ax->mem.device = dev;
  Axis1D& h = ax->host;
  if (!build_axis(kind, n, faces, loc, lo, hi, h).empty()) return HELM_EINVAL;
  if (h.m > 512) return HELM_EINVAL;
  if (!eigen_1d(h).empty()) return HELM_EINVAL;
  const int m = h.m;
  std::vector<double> coef(3 * m);
  for (int i = 0; i < m; ++i) {
    coef[3 * i] = h.lower[i];
    coef[3 * i + 1] = h.diag[i];
    coef[3 * i + 2] = h.upper[i];
  }
  hipError_t e = hipSuccess;
  DevBlocks& mem = ax->mem;
  if (e == hipSuccess) e = mem.upload(&ax->lam, h.lam.data(), m);
  if (e == hipSuccess) e = mem.upload(&ax->coef, coef.data(), coef.size());
  if (e == hipSuccess) e = mem.upload(&ax->kdiag, h.k_diag.data(), m);
  if (e == hipSuccess) e = mem.upload(&ax->koff, h.k_off.data(), h.k_off.size());
  if (e == hipSuccess) e = mem.upload(&ax->vol, h.vol.data(), m);
  if (e == hipSuccess) e = mem.upload(&ax->E, h.E.data(), h.E.size());
  if (e == hipSuccess) e = mem.upload(&ax->Einv, h.Einv.data(), h.Einv.size());
  if (e == hipSuccess) {  // fast transform tables of a uniform axis
    int sine = 0, M = 0;
    double alpha = 0.0, beta = 0.0;
    FftHost hf, hi;
    if (fft_axis_params(h, sine, alpha, beta, M) && fft_plan(sine, alpha, beta, M, m, true, hf) &&
        fft_plan(sine, alpha, beta, M, m, false, hi)) {
      double* W = nullptr;
      double* pf[2] = {nullptr, nullptr};
      double* pi[2] = {nullptr, nullptr};
      e = mem.upload(&W, hf.W.data(), hf.W.size());
      if (e == hipSuccess) e = mem.upload(&pf[0], hf.pre.data(), hf.pre.size());
      if (e == hipSuccess) e = mem.upload(&pf[1], hf.post.data(), hf.post.size());
      if (e == hipSuccess) e = mem.upload(&pi[0], hi.pre.data(), hi.pre.size());
      if (e == hipSuccess) e = mem.upload(&pi[1], hi.post.data(), hi.post.size());
      const FftHost* hs[2] = {&hf, &hi};
      double* const* ps[2] = {pf, pi};
      for (int dir = 0; dir < 2; ++dir) {
        FftTables& t = ax->fft[dir];
        t.L = hs[dir]->L;
        t.N = hs[dir]->N;
        t.M = hs[dir]->M;
        t.nst = hs[dir]->nst;
        t.lines = hs[dir]->lines;
        t.refl = hs[dir]->refl;
        for (int q = 0; q < t.nst; ++q) t.rad[q] = hs[dir]->rad[q];
        t.W = W;
        t.pre = ps[dir][0];
        t.post = ps[dir][1];
      }
      ax->fft_ok = e == hipSuccess;
    }
  }
  if (e == hipSuccess && !h.gdiag.empty()) e = mem.upload(&ax->gdiag, h.gdiag.data(), h.gdiag.size());
  if (e == hipSuccess && !h.inv_r2.empty()) e = mem.upload(&ax->inv_r2, h.inv_r2.data(), h.inv_r2.size());
  for (int p = 0; p < 3 && e == hipSuccess; ++p) {
    const Prec pr = static_cast<Prec>(p);
    const size_t bytes = swizzled_bytes(pr, m);
    std::vector<unsigned char> buf(bytes);
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
      swizzle_operand(pr, m, dir == 0 ? h.Einv.data() : h.E.data(), buf.data());
      e = mem.upload(reinterpret_cast<unsigned char**>(&ax->sw[p][dir]), buf.data(), bytes);
    }
  }
  if (e == hipSuccess) {
    const size_t bytes = swizzled_bf16x3_bytes(m);
    std::vector<unsigned char> buf(bytes);
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
      swizzle_bf16x3(m, dir == 0 ? h.Einv.data() : h.E.data(), buf.data());
      e = mem.upload(reinterpret_cast<unsigned char**>(&ax->sw3[dir]), buf.data(), bytes);
    }
  }
  if (e != hipSuccess) return from_hip(e);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      auto existing = it->second.lock();
      if (existing) {
        out = existing;
        return HELM_OK;
      }
    }
    if (g_cache.size() >= 1024) purge_expired(g_cache);
    g_cache[key] = ax;
  }
  out = ax;
  return HELM_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device buffer freed (on its device) with its last owner.
struct DevBuf {
  double* p = nullptr;
  DevBlocks mem;
};

// lambda_x[a] + lambda_y[b] per (x axis, y axis) pair, summed in FP64 and shared by every plan
// on that pair (the per-(a, b) part of the eq. 26-27 denominator for split-BF16 solves), so
// that building or dropping a plan on cached axes touches no device memory.
std::mutex g_pair_mu;
std::map<std::string, std::weak_ptr<DevBuf>> g_pair_cache;

// The three axes of a plan into ax[0..2]: axis(d, build) is get_axis for plan axis d.  Axes
// in the cache are taken first; the missing ones (each an eigen-decomposition on the host) are
// built concurrently, one on the caller's thread and the others on threads of their own that
// take the caller's device.  Returns the first failure in axis order.
template <typename F>
helm_status get_axes(std::shared_ptr<DevAxis>* ax, F&& axis) {
  helm_status st[3] = {HELM_OK, HELM_OK, HELM_OK};
  int miss[3], nmiss = 0;
  for (int d = 0; d < 3; ++d) {
    if ((st[d] = axis(d, false)) != HELM_OK) return st[d];
    if (!ax[d]) miss[nmiss++] = d;
  }
  if (nmiss == 0) return HELM_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HELM_EDEVICE;
  std::vector<std::thread> pool;
  for (int q = 1; q < nmiss; ++q) {
    const int d = miss[q];
    try {
      pool.emplace_back([&, d] { st[d] = hipSetDevice(dev) == hipSuccess ? axis(d, true) : HELM_EDEVICE; });
    } catch (const std::system_error&) {  // no thread to be had: built on the caller's
      st[d] = axis(d, true);
    }
  }
  st[miss[0]] = axis(miss[0], true);
  for (auto& t : pool) t.join();
  for (helm_status x : st)
    if (x != HELM_OK) return x;
  return HELM_OK;
}

helm_status get_lamxy(const DevAxis& X, const DevAxis& Y, std::shared_ptr<DevBuf>& out) {
  const std::string key = X.key + "|" + Y.key;
  std::lock_guard<std::mutex> lk(g_pair_mu);
  auto it = g_pair_cache.find(key);
  if (it != g_pair_cache.end() && (out = it->second.lock())) return HELM_OK;
  const int mx = X.host.m, my = Y.host.m;
  std::vector<double> t(static_cast<size_t>(mx) * my);
  for (int b = 0; b < my; ++b)
    for (int a = 0; a < mx; ++a) t[static_cast<size_t>(b) * mx + a] = X.host.lam[a] + Y.host.lam[b];
  auto buf = std::make_shared<DevBuf>();
  buf->mem.device = X.device;
  buf->mem.alloc = X.mem.alloc;
  const hipError_t e = buf->mem.upload(&buf->p, t.data(), t.size());
  if (e != hipSuccess) return from_hip(e);
  if (g_pair_cache.size() >= 1024) purge_expired(g_pair_cache);
  g_pair_cache[key] = buf;
  out = buf;
  return HELM_OK;
}

// Pinned host buffers for the refinement norms (2 * kMaxRhs * kNormStripes words each), taken
// by a solve for its duration and returned: the pool grows to the peak number of concurrent
// refined solves and lives until process exit (pinned allocation and release synchronize the
// device, so they stay off the solve path).
std::mutex g_pin_mu;
std::vector<unsigned long long*> g_pin_pool;

unsigned long long* take_pinned_norms() {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin_pool.empty()) {
      unsigned long long* b = g_pin_pool.back();
      g_pin_pool.pop_back();
      return b;
    }
  }
  unsigned long long* b = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&b), 2 * kMaxRhs * kNormStripes * sizeof(unsigned long long)) !=
      hipSuccess)
    return nullptr;
  return b;
}
void give_pinned_norms(unsigned long long* b) {
  if (!b) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_pool.push_back(b);
}
struct PinnedNorms {
  unsigned long long* p = take_pinned_norms();
  ~PinnedNorms() { give_pinned_norms(p); }
};

}  // namespace

namespace helm {
hipError_t wait_stream(hipStream_t st) {
  struct ThreadEvent {
    int device = -1;
    hipEvent_t ev = nullptr;
    ~ThreadEvent() {
      if (ev) (void)hipEventDestroy(ev);
    }
  };
  thread_local ThreadEvent te;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (te.device != dev) {
    if (te.ev) (void)hipEventDestroy(te.ev);
    te.ev = nullptr;
    te.device = -1;
    if ((e = hipEventCreateWithFlags(&te.ev, hipEventDisableTiming)) != hipSuccess) return e;
    te.device = dev;
  }
  if ((e = hipEventRecord(te.ev, st)) != hipSuccess) return e;
  while ((e = hipEventQuery(te.ev)) == hipErrorNotReady) std::this_thread::yield();
  return e;
}
}  // namespace helm

// Optional per-launch event timing (helm_profile_enable / helm_profile_read).
struct StageProfiler {
  bool on = false;
  unsigned mask = ~0u;  // stages timed when on
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      // timing only: no system-scope fence (a cache writeback and invalidate) at each record
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void clear() {
    recs.clear();
    used = 0;
  }
  ~StageProfiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct helm_plan {
  std::shared_ptr<DevAxis> ax[3];
  int m[3] = {0, 0, 0};   // unknowns per axis
  double sigma = 0.0;
  helm_opts opts{};
  bool all_neumann = false;
  bool cyl = false;       // cylindrical operator (x = theta, y = z, z = r): FP64, Thomas along r
  int device = 0;
  std::shared_ptr<DevBuf> lamxy;             // m[0] * m[1]: lamx[a] + lamy[b] (split-BF16), shared
  mutable StageProfiler prof;
  long long npts() const { return static_cast<long long>(m[0]) * m[1] * m[2]; }
  // The Thomas form (FP64): TPT_Z plans and every cylindrical plan.  The workspace layout and the
  // solve dispatch both use this, so a Thomas solve always has its checkpoint region.
  bool thomas() const { return cyl || opts.method == HELM_TPT_Z; }
  bool refined() const {
    return opts.precision == HELM_FP32_IR || opts.precision == HELM_BF16_IR || opts.precision == HELM_BF16X3_IR;
  }
  Prec prec() const {
    switch (opts.precision) {
      case HELM_FP32:
      case HELM_FP32_IR: return P_F32;
      case HELM_BF16:
      case HELM_BF16_IR: return P_BF16;
      case HELM_BF16X3:
      case HELM_BF16X3_IR: return P_BF16X3;
      default: return P_F64;
    }
  }
};

extern "C" {

void helm_default_opts(helm_opts* o) {
  if (!o) return;
  o->precision = HELM_FP64;
  o->method = HELM_TPF;
  o->ir_tol = 1e-11;
  o->max_sweeps = 12;
  o->null_mode = HELM_NULL_PROJECT;
  o->alloc = nullptr;
  o->dealloc = nullptr;
  o->alloc_ctx = nullptr;
}

const char* helm_status_str(helm_status s) {
  switch (s) {
    case HELM_OK: return "HELM_OK";
    case HELM_EINVAL: return "HELM_EINVAL: invalid argument";
    case HELM_ESINGULAR: return "HELM_ESINGULAR: zero denominator outside the Neumann null mode";
    case HELM_ENOMEM: return "HELM_ENOMEM: out of memory";
    case HELM_EDEVICE: return "HELM_EDEVICE: HIP runtime error";
    case HELM_ENOTCONVERGED: return "HELM_ENOTCONVERGED: tolerance not reached";
    case HELM_ENONFINITE: return "HELM_ENONFINITE: NaN or Inf encountered";
  }
  return "unknown helm_status";
}

helm_status helm_host_operator_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi, int* m_out,
                                  double* lower, double* diag, double* upper, double* vol) {
  Axis1D ax;
  if (!build_operator_1d(n, faces, loc, bc_lo, bc_hi, ax).empty()) return HELM_EINVAL;
  if (m_out) *m_out = ax.m;
  if (lower) std::copy(ax.lower.begin(), ax.lower.end(), lower);
  if (diag) std::copy(ax.diag.begin(), ax.diag.end(), diag);
  if (upper) std::copy(ax.upper.begin(), ax.upper.end(), upper);
  if (vol) std::copy(ax.vol.begin(), ax.vol.end(), vol);
  return HELM_OK;
}

helm_status helm_host_eigen_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi, int* m_out, double* lam,
                               double* E, double* Einv) {
  Axis1D ax;
  if (!build_operator_1d(n, faces, loc, bc_lo, bc_hi, ax).empty()) return HELM_EINVAL;
  if (!eigen_1d(ax).empty()) return HELM_EINVAL;
  if (m_out) *m_out = ax.m;
  if (lam) std::copy(ax.lam.begin(), ax.lam.end(), lam);
  if (E) std::copy(ax.E.begin(), ax.E.end(), E);
  if (Einv) std::copy(ax.Einv.begin(), ax.Einv.end(), Einv);
  return HELM_OK;
}

static bool valid_opts(const helm_opts& o) {
  if (o.precision < HELM_FP64 || o.precision > HELM_BF16X3_IR) return false;
  if (o.method != HELM_TPF && o.method != HELM_TPT_Z && o.method != HELM_FFT) return false;
  if (o.null_mode != HELM_NULL_PROJECT && o.null_mode != HELM_NULL_PAPER_EQ28) return false;
  if (!(o.ir_tol >= 0.0) || o.max_sweeps < 1) return false;
  if (!DevAlloc::from(o).valid()) return false;
  // The Thomas and fast-transform paths run in FP64 only.
  if ((o.method == HELM_TPT_Z || o.method == HELM_FFT) && o.precision != HELM_FP64) return false;
  return true;
}

// Is some denominator lam_x + lam_y + lam_z + sigma numerically zero, other than the exact
// all-Neumann null mode?  Only reachable with sigma < 0 (all eigenvalues are >= 0).
static bool has_zero_denominator(const helm_plan* p, double sigma) {
  if (sigma >= 0.0) return false;
  const auto& lx = p->ax[0]->host.lam;
  const auto& ly = p->ax[1]->host.lam;
  const auto& lz = p->ax[2]->host.lam;
  const double scale = lx.back() + ly.back() + lz.back() + std::fabs(sigma);
  for (double c : lz)
    for (double b : ly)
      for (double a : lx)
        if (std::fabs(a + b + c + sigma) <= 1e-13 * scale) return true;
  return false;
}

helm_status helm_setup(const helm_grid* grid, const helm_bc* bc, double sigma, const helm_opts* opts,
                       helm_plan** out) {
  if (!grid || !bc || !out) return HELM_EINVAL;
  *out = nullptr;
  if (!std::isfinite(sigma)) return HELM_EINVAL;
  helm_opts o;
  helm_default_opts(&o);
  if (opts) o = *opts;
  if (!valid_opts(o)) return HELM_EINVAL;
  std::unique_ptr<helm_plan> p(new (std::nothrow) helm_plan());
  if (!p) return HELM_ENOMEM;
  p->opts = o;
  p->sigma = sigma;
  if (hipGetDevice(&p->device) != hipSuccess) return HELM_EDEVICE;
  for (int d = 0; d < 3; ++d)
    if (!grid->faces[d]) return HELM_EINVAL;
  const DevAlloc al = DevAlloc::from(o);
  const helm_status sa = get_axes(p->ax, [&](int d, bool build) {
    return get_axis(AXIS_CART, grid->n[d], grid->faces[d], grid->loc[d], bc->lo[d], bc->hi[d], al, p->ax[d], build);
  });
  if (sa != HELM_OK) return sa;
  bool alln = true;
  for (int d = 0; d < 3; ++d) {
    p->m[d] = p->ax[d]->host.m;
    alln = alln && p->ax[d]->host.null_mode;
  }
  p->all_neumann = alln;
  if (has_zero_denominator(p.get(), sigma)) return HELM_ESINGULAR;
  if (p->prec() == P_BF16X3) {
    const helm_status s = get_lamxy(*p->ax[0], *p->ax[1], p->lamxy);
    if (s != HELM_OK) return s;
  }
  *out = p.release();
  return HELM_OK;
}

helm_status helm_cyl_setup(const helm_cyl_grid* grid, const helm_bc* bc, double sigma, const helm_opts* opts,
                           helm_plan** out) {
  if (!grid || !bc || !out) return HELM_EINVAL;
  *out = nullptr;
  if (!std::isfinite(sigma) || sigma < 0.0) return HELM_EINVAL;
  helm_opts o;
  helm_default_opts(&o);
  if (opts) o = *opts;
  o.method = HELM_TPT_Z;  // eq. 44: transforms in theta and z, one Thomas solve per radial line
  if (o.precision != HELM_FP64 || !valid_opts(o)) return HELM_EINVAL;
  if (grid->theta_periodic != 0 && grid->theta_periodic != 1) return HELM_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!grid->faces[d]) return HELM_EINVAL;
  std::unique_ptr<helm_plan> p(new (std::nothrow) helm_plan());
  if (!p) return HELM_ENOMEM;
  p->opts = o;
  p->sigma = sigma;
  p->cyl = true;
  if (hipGetDevice(&p->device) != hipSuccess) return HELM_EDEVICE;
  const DevAlloc al = DevAlloc::from(o);
  // plan axes: x = theta (fastest), y = z, z = r (slowest: the Thomas direction)
  const helm_status s = get_axes(p->ax, [&](int d, bool build) {
    if (d == 0)
      return grid->theta_periodic
                 ? get_axis(AXIS_PERIODIC, grid->n[1], grid->faces[1], HELM_CELL, 1, 1, al, p->ax[0], build)
                 : get_axis(AXIS_CART, grid->n[1], grid->faces[1], HELM_CELL, bc->lo[1], bc->hi[1], al, p->ax[0],
                            build);
    if (d == 1)
      return get_axis(AXIS_CART, grid->n[2], grid->faces[2], HELM_CELL, bc->lo[2], bc->hi[2], al, p->ax[1], build);
    return get_axis(AXIS_RADIAL, grid->n[0], grid->faces[0], HELM_CELL, bc->lo[0], bc->hi[0], al, p->ax[2], build);
  });
  if (s != HELM_OK) return s;
  bool alln = true;
  for (int d = 0; d < 3; ++d) {
    p->m[d] = p->ax[d]->host.m;
    alln = alln && p->ax[d]->host.null_mode;
  }
  p->all_neumann = alln;
  *out = p.release();
  return HELM_OK;
}

helm_status helm_host_operator_cyl(int kind, int n, const double* faces, int bc_lo, int bc_hi, int* m_out,
                                   double* lower, double* diag, double* upper, double* vol) {
  if (kind != 0 && kind != 1) return HELM_EINVAL;
  Axis1D ax;
  if (!build_axis(kind == 0 ? AXIS_RADIAL : AXIS_PERIODIC, n, faces, HELM_CELL, bc_lo, bc_hi, ax).empty())
    return HELM_EINVAL;
  if (m_out) *m_out = ax.m;
  if (lower) std::copy(ax.lower.begin(), ax.lower.end(), lower);
  if (diag) std::copy(ax.diag.begin(), ax.diag.end(), diag);
  if (upper) std::copy(ax.upper.begin(), ax.upper.end(), upper);
  if (vol) std::copy(ax.vol.begin(), ax.vol.end(), vol);
  return HELM_OK;
}

helm_status helm_host_eigen_cyl(int kind, int n, const double* faces, int bc_lo, int bc_hi, int* m_out, double* lam,
                                double* E, double* Einv) {
  if (kind != 0 && kind != 1) return HELM_EINVAL;
  Axis1D ax;
  if (!build_axis(kind == 0 ? AXIS_RADIAL : AXIS_PERIODIC, n, faces, HELM_CELL, bc_lo, bc_hi, ax).empty())
    return HELM_EINVAL;
  if (!eigen_1d(ax).empty()) return HELM_EINVAL;
  if (m_out) *m_out = ax.m;
  if (lam) std::copy(ax.lam.begin(), ax.lam.end(), lam);
  if (E) std::copy(ax.E.begin(), ax.E.end(), E);
  if (Einv) std::copy(ax.Einv.begin(), ax.Einv.end(), Einv);
  return HELM_OK;
}

// Workspace layout (each region 256-byte aligned):
//   FP64:  W    nrhs*P doubles         (+ Thomas checkpoints for TPT_Z)
//   low :  L1, L2  nrhs*P low-precision values each (split-BF16 with refinement: also L3, the
//          first solve in FP32), norms 2*nrhs u64
static void workspace_layout(const helm_plan* p, int nrhs, size_t* total, size_t* off_a, size_t* off_b,
                             size_t* off_norms, size_t* off_mean = nullptr, size_t* off_c = nullptr) {
  const size_t P = static_cast<size_t>(p->npts()) * nrhs;
  size_t t = 0;
  if (p->prec() == P_F64) {
    *off_a = 0;
    t = align_up(P * 8, 256);
    *off_b = t;
    if (p->thomas()) t += align_up(thomas_scratch_bytes(p->m[0], p->m[1], p->m[2], nrhs), 256);
    *off_norms = t;
  } else {
    const size_t es = p->prec() == P_BF16 ? 2 : 4;
    *off_a = 0;
    t = align_up(P * es, 256);
    *off_b = t;
    t += align_up(P * es, 256);
    if (off_c) *off_c = t;
    if (p->prec() == P_BF16X3 && p->refined()) t += align_up(P * 4, 256);
    *off_norms = t;
    t += align_up(2 * kMaxRhs * kNormStripes * sizeof(unsigned long long), 256);
  }
  if (off_mean) *off_mean = t;
  if (p->all_neumann) t += align_up(static_cast<size_t>(nrhs) * (kMeanBlocks + 1) * sizeof(double), 256);
  *total = t;
}

helm_status helm_workspace_size(const helm_plan* p, int nrhs, size_t* bytes) {
  if (!p || !bytes || nrhs < 1 || nrhs > kMaxRhs) return HELM_EINVAL;
  size_t a, b, c;
  workspace_layout(p, nrhs, bytes, &a, &b, &c);
  return HELM_OK;
}

helm_status helm_get_eigen(const helm_plan* p, int axis, int* n, double* lam, double* E, double* Einv) {
  if (!p || axis < 0 || axis > 2) return HELM_EINVAL;
  const Axis1D& h = p->ax[axis]->host;
  if (n) *n = h.m;
  if (lam) std::copy(h.lam.begin(), h.lam.end(), lam);
  if (E) std::copy(h.E.begin(), h.E.end(), E);
  if (Einv) std::copy(h.Einv.begin(), h.Einv.end(), Einv);
  return HELM_OK;
}

void helm_destroy(helm_plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  (void)hipSetDevice(cur);
  delete p;
}

}  // extern "C"

void helm::release_plan(helm_plan* p) { delete p; }

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename F>
hipError_t timed(const helm_plan* p, int stage, hipStream_t st, F&& launch) {
  if (!p->prof.on || !((p->prof.mask >> stage) & 1u)) return launch();
  hipEvent_t a = p->prof.take(), b = p->prof.take();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  if (e == hipSuccess) p->prof.recs.push_back({stage, a, b});
  return e;
}

// Six mode products of one TPF application in precision pr, from `in` (type pr) to the
// final x-inverse output.  bufs: two scratch buffers of type pr; the final product writes
// `out` with epilogue epi_last (STORE in pr, or ACCUM into FP64 u).
hipError_t tpf_products(const helm_plan* p, Prec pr, const void* in, void* b1, void* b2, void* out, Epi epi_last,
                        int nrhs, const double* sig, unsigned long long* norms, int accum_zero, hipStream_t st,
                        bool in_f64 = false, bool u0_f32 = false, const float* u0 = nullptr,
                        const GroupTabs* grp = nullptr) {
  const DevAxis& X = *p->ax[0];
  const DevAxis& Y = *p->ax[1];
  const DevAxis& Z = *p->ax[2];
  const long long nx = p->m[0], ny = p->m[1], nz = p->m[2];
  EpiArgs ep;
  ep.lamx = X.lam;
  ep.lamy = Y.lam;
  ep.lamz = Z.lam;
  ep.lamxy = p->lamxy ? p->lamxy->p : nullptr;
  ep.nx = static_cast<int>(nx);
  ep.eq28 = p->opts.null_mode == HELM_NULL_PAPER_EQ28;
  ep.norms = norms;
  ep.rows_per_rhs = ny * nz;
  ep.accum_zero = accum_zero;
  for (int r = 0; r < nrhs; ++r) ep.sigma[r] = sig[r];
  if (grp) {
    ep.lamx_rhs = grp->lam[0];
    ep.lamy_rhs = grp->lam[1];
    ep.lamz_rhs = grp->lam[2];
    ep.lamxy_rhs = grp->lamxy;
  }
  // the arguments of one stage: in a grouped solve, the per-RHS operand of (axis, direction)
  // and the extent of one RHS in the stage's tiled dimension
  auto G = [&](int axis, int dir, long long span) -> const EpiArgs& {
    if (grp) {
      ep.msw_rhs = grp->msw[axis][dir];
      ep.span = span;
    }
    return ep;
  };
  hipError_t e;
  if (pr == P_BF16X3) {
    // rotating layout: [k][j][i] -> [a][k][j] -> [b][a][k] -> [c][b][a] -> [i][c][b] -> [j][i][c] -> [k][j][i]
    float* f1 = static_cast<float*>(b1);
    float* f2 = static_cast<float*>(b2);
    if ((e = timed(p, in_f64 ? HELM_STAGE_X_FWD_RHS : HELM_STAGE_X_FWD, st, [&] {
           return mode_rot(X.sw3[0], nx, in, in_f64, f1, nrhs, ny * nz, EPI_STORE, G(0, 0, ny * nz), st);
         })) != hipSuccess)
      return e;
    if ((e = timed(p, HELM_STAGE_Y_FWD, st, [&] {
           return mode_rot(Y.sw3[0], ny, f1, false, f2, nrhs, nz * nx, EPI_STORE, G(1, 0, nz * nx), st);
         })) != hipSuccess)
      return e;
    if ((e = timed(p, HELM_STAGE_Z_FWD_DIV, st, [&] {
           return mode_rot(Z.sw3[0], nz, f2, false, f1, nrhs, nx * ny, EPI_DIVIDE, G(2, 0, nx * ny), st);
         })) != hipSuccess)
      return e;
    if ((e = timed(p, HELM_STAGE_X_INV, st, [&] {
           return mode_rot(X.sw3[1], nx, f1, false, f2, nrhs, nz * ny, EPI_STORE, G(0, 1, nz * ny), st);
         })) != hipSuccess)
      return e;
    if ((e = timed(p, HELM_STAGE_Y_INV, st, [&] {
           return mode_rot(Y.sw3[1], ny, f2, false, f1, nrhs, nx * nz, EPI_STORE, G(1, 1, nx * nz), st);
         })) != hipSuccess)
      return e;
    if (epi_last != EPI_ACCUM) return hipErrorInvalidValue;
    if (accum_zero) {
      // first solve (u = 0): the product writes u directly, in FP64 as the result, or in FP32
      // (u0_f32) when refinement follows: its error (~1e-7) is far above FP32 rounding, and the
      // FP64 residual of the FP32 values is exact, so the next sweep corrects both
      return timed(p, HELM_STAGE_Z_INV_U, st, [&] {
        return mode_rot(Z.sw3[1], nz, f1, false, out, nrhs, ny * nx, u0_f32 ? EPI_STORE : EPI_STORE_F64, G(2, 1, ny * nx),
                        st);
      });
    }
    // a correction lands in FP32 (natural layout) and is added to u by a streaming kernel
    // that also takes the norms the refinement loop stops on
    if ((e = timed(p, HELM_STAGE_Z_INV, st, [&] {
           return mode_rot(Z.sw3[1], nz, f1, false, f2, nrhs, ny * nx, EPI_STORE, G(2, 1, ny * nx), st);
         })) != hipSuccess)
      return e;
    // u = u0 + du when the previous iterate is the FP32 first solve, else u += du
    return timed(p, HELM_STAGE_UPDATE, st, [&] {
      return update_u(static_cast<double*>(out), f2, nx * ny * nz, nrhs, 0, norms, st, u0);
    });
  }
  const int ip = static_cast<int>(pr);
  // HELM_FFT (FP64): uniform axes by fast sine/cosine transforms, the rest by the products
  const bool fast = pr == P_F64 && p->opts.method == HELM_FFT;
  const bool fx = fast && X.fft_ok, fy = fast && Y.fft_ok, fz = fast && Z.fft_ok;
  const long long P3 = nx * ny * nz;
  FftLines lx, ly, lz;  // lines along x (contiguous), y and z (strided) of all right-hand sides
  lx.nlines = nrhs * nz * ny;
  lx.n0 = ny;
  lx.n1 = nz;
  lx.t0 = nx;
  lx.t1 = nx * ny;
  lx.t2 = P3;
  lx.se = 1;
  ly.nlines = nrhs * nz * nx;
  ly.n0 = nx;
  ly.n1 = nz;
  ly.t0 = 1;
  ly.t1 = nx * ny;
  ly.t2 = P3;
  ly.se = nx;
  lz.nlines = nrhs * ny * nx;
  lz.n0 = nx;
  lz.n1 = ny;
  lz.t0 = 1;
  lz.t1 = nx;
  lz.t2 = P3;
  lz.se = nx * ny;
  // forward: E_x^{-1}, E_y^{-1}, E_z^{-1} + divide
  if ((e = timed(p, HELM_STAGE_X_FWD, st, [&] {
         if (fx) return fft_axis(static_cast<const double*>(in), static_cast<double*>(b1), X.fft[0], lx, EPI_STORE, ep, st);
         return mode_right(pr, X.sw[ip][0], nx, in, pr, b1, pr, nrhs * ny * nz, EPI_STORE, G(0, 0, ny * nz), st);
       })) != hipSuccess)
    return e;
  if ((e = timed(p, HELM_STAGE_Y_FWD, st, [&] {
         if (fy) return fft_axis(static_cast<const double*>(b1), static_cast<double*>(b2), Y.fft[0], ly, EPI_STORE, ep, st);
         return mode_left(pr, Y.sw[ip][0], ny, b1, pr, b2, pr, nrhs * nz, nx, EPI_STORE, G(1, 0, nz * nx), st);
       })) != hipSuccess)
    return e;
  if ((e = timed(p, HELM_STAGE_Z_FWD_DIV, st, [&] {
         if (fz) return fft_axis(static_cast<const double*>(b2), static_cast<double*>(b1), Z.fft[0], lz, EPI_DIVIDE, ep, st);
         return mode_left(pr, Z.sw[ip][0], nz, b2, pr, b1, pr, nrhs, nx * ny, EPI_DIVIDE, G(2, 0, nx * ny), st);
       })) != hipSuccess)
    return e;
  // inverse: E_z, E_y, E_x
  if ((e = timed(p, HELM_STAGE_Z_INV, st, [&] {
         if (fz) return fft_axis(static_cast<const double*>(b1), static_cast<double*>(b2), Z.fft[1], lz, EPI_STORE, ep, st);
         return mode_left(pr, Z.sw[ip][1], nz, b1, pr, b2, pr, nrhs, nx * ny, EPI_STORE, G(2, 1, nx * ny), st);
       })) != hipSuccess)
    return e;
  if ((e = timed(p, HELM_STAGE_Y_INV, st, [&] {
         if (fy) return fft_axis(static_cast<const double*>(b2), static_cast<double*>(b1), Y.fft[1], ly, EPI_STORE, ep, st);
         return mode_left(pr, Y.sw[ip][1], ny, b2, pr, b1, pr, nrhs * nz, nx, EPI_STORE, G(1, 1, nz * nx), st);
       })) != hipSuccess)
    return e;
  const Prec tout = epi_last == EPI_ACCUM ? P_F64 : pr;
  return timed(p, HELM_STAGE_X_INV, st, [&] {
    if (fx && epi_last == EPI_STORE)
      return fft_axis(static_cast<const double*>(b1), static_cast<double*>(out), X.fft[1], lx, EPI_STORE, ep, st);
    return mode_right(pr, X.sw[ip][1], nx, b1, pr, out, tout, nrhs * ny * nz, epi_last, G(0, 1, ny * nz), st);
  });
}

StencilArgs stencil_args(const helm_plan* p, int nrhs, const double* sig, const GroupTabs* grp = nullptr) {
  StencilArgs a;
  a.cx = p->ax[0]->coef;
  a.cy = p->ax[1]->coef;
  a.cz = p->ax[2]->coef;
  if (grp) {
    a.cx_rhs = grp->coef[0];
    a.cy_rhs = grp->coef[1];
    a.cz_rhs = grp->coef[2];
  }
  a.nx = p->m[0];
  a.ny = p->m[1];
  a.nz = p->m[2];
  a.nrhs = nrhs;
  a.xscale = p->cyl ? p->ax[2]->inv_r2 : nullptr;
  a.xper = p->ax[0]->host.periodic ? 1 : 0;
  for (int r = 0; r < nrhs; ++r) a.sigma[r] = sig[r];
  return a;
}

}  // namespace

extern "C" helm_status helm_apply(const helm_plan* p, const double* u, double* Hu, int nrhs,
                                  const double* sigma_per_rhs, void* stream) {
  if (!p || !u || !Hu || nrhs < 1 || nrhs > kMaxRhs || u == Hu) return HELM_EINVAL;
  double sig[kMaxRhs];
  for (int r = 0; r < nrhs; ++r) {
    sig[r] = sigma_per_rhs ? sigma_per_rhs[r] : p->sigma;
    if (!std::isfinite(sig[r])) return HELM_EINVAL;
  }
  DeviceGuard dg(p->device);
  const StencilArgs a = stencil_args(p, nrhs, sig);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return from_hip(timed(p, HELM_STAGE_APPLY, st, [&] { return stencil(0, u, nullptr, Hu, P_F64, a, st); }));
}

extern "C" helm_status helm_solve(helm_plan* p, const double* f, double* u, int nrhs, const double* sigma_per_rhs,
                                  void* ws, void* stream, helm_info* info) {
  return helm::solve_impl(p, f, u, nrhs, sigma_per_rhs, ws, stream, info, false);
}

int helm::plan_device(const helm_plan* p) { return p ? p->device : -1; }

// ---------------------------------------------------------------- grouped solves
namespace {

// Pointer slots of a grouped solve's device table: msw[axis][dir] (6), lam[axis] (3), lamxy,
// coef[axis] (3), kMaxRhs entries each.
constexpr int kGroupSlots = 13;
constexpr size_t kGroupTabBytes = static_cast<size_t>(kGroupSlots) * kMaxRhs * sizeof(void*);

// Checks that the plans can share one solve and returns the total right-hand-side count.
helm_status group_check(helm_plan* const* plans, int nplans, const int* nrhs, int* total) {
  if (!plans || !nrhs || nplans < 1 || !total) return HELM_EINVAL;
  const helm_plan* p0 = plans[0];
  if (!p0) return HELM_EINVAL;
  int t = 0;
  for (int i = 0; i < nplans; ++i) {
    const helm_plan* q = plans[i];
    if (!q || nrhs[i] < 1) return HELM_EINVAL;
    t += nrhs[i];
    if (t > kMaxRhs) return HELM_EINVAL;
    if (q->cyl || q->opts.method != HELM_TPF || (q->prec() != P_F64 && q->prec() != P_BF16X3)) return HELM_EINVAL;
    if (q->device != p0->device || q->opts.precision != p0->opts.precision || q->opts.ir_tol != p0->opts.ir_tol ||
        q->opts.max_sweeps != p0->opts.max_sweeps || q->opts.null_mode != p0->opts.null_mode)
      return HELM_EINVAL;
    for (int d = 0; d < 3; ++d)
      if (q->m[d] != p0->m[d]) return HELM_EINVAL;
  }
  *total = t;
  return HELM_OK;
}

size_t group_tab_offset(const helm_plan* p0, int total) {
  size_t bytes = 0, a, b, c;
  workspace_layout(p0, total, &bytes, &a, &b, &c);
  return align_up(bytes, 256);
}

}  // namespace

bool helm::plans_groupable(const helm_plan* a, const helm_plan* b) {
  if (!a || !b) return false;
  helm_plan* const pl[2] = {const_cast<helm_plan*>(a), const_cast<helm_plan*>(b)};
  const int n[2] = {1, 1};
  int total = 0;
  if (group_check(pl, 2, n, &total) != HELM_OK) return false;
  const long long nx = a->m[0], ny = a->m[1], nz = a->m[2];
  return (ny * nz) % 512 == 0 && (nz * nx) % 512 == 0 && (nx * ny) % 512 == 0;
}

extern "C" helm_status helm_group_workspace_size(helm_plan* const* plans, int nplans, const int* nrhs,
                                                 size_t* bytes) {
  int total = 0;
  if (!bytes) return HELM_EINVAL;
  const helm_status s = group_check(plans, nplans, nrhs, &total);
  if (s != HELM_OK) return s;
  *bytes = group_tab_offset(plans[0], total) + kGroupTabBytes;
  return HELM_OK;
}

extern "C" helm_status helm_solve_group(helm_plan* const* plans, int nplans, const int* nrhs, const double* f,
                                        double* u, const double* sigma, void* ws, void* stream, helm_info* info) {
  int total = 0;
  helm_status s = group_check(plans, nplans, nrhs, &total);
  if (s != HELM_OK) return s;
  if (!f || !u || !ws) return HELM_EINVAL;
  helm_plan* p0 = plans[0];
  std::vector<double> sig(total);
  std::vector<const helm_plan*> owner(total);
  bool one_plan = true;
  for (int i = 0, r = 0; i < nplans; ++i) {
    one_plan = one_plan && plans[i] == p0;
    for (int k = 0; k < nrhs[i]; ++k, ++r) {
      sig[r] = sigma ? sigma[r] : plans[i]->sigma;
      owner[r] = plans[i];
    }
  }
  // one plan: an ordinary multi-RHS solve
  if (one_plan) return helm::solve_impl(p0, f, u, total, sig.data(), ws, stream, info, false);
  // the per-RHS table, written into the workspace by the stream itself
  std::vector<const void*> tab(static_cast<size_t>(kGroupSlots) * kMaxRhs, nullptr);
  const int ip = static_cast<int>(p0->prec());
  for (int r = 0; r < total; ++r) {
    const helm_plan* q = owner[r];
    for (int a = 0; a < 3; ++a) {
      const DevAxis& A = *q->ax[a];
      for (int d = 0; d < 2; ++d)
        tab[(2 * a + d) * kMaxRhs + r] = ip == P_BF16X3 ? A.sw3[d] : A.sw[ip][d];
      tab[(6 + a) * kMaxRhs + r] = A.lam;
      tab[(10 + a) * kMaxRhs + r] = A.coef;
    }
    tab[9 * kMaxRhs + r] = q->lamxy ? q->lamxy->p : nullptr;
    if (ip == P_BF16X3 && !q->lamxy) return HELM_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return HELM_EINVAL;
  const void** dtab =
      reinterpret_cast<const void**>(static_cast<unsigned char*>(ws) + group_tab_offset(p0, total));
  DeviceGuard dg(p0->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (helm::write_ptrs(tab.data(), static_cast<int>(tab.size()), dtab, st) != hipSuccess) return HELM_EDEVICE;
  helm::GroupTabs g;
  for (int a = 0; a < 3; ++a) {
    for (int d = 0; d < 2; ++d) g.msw[a][d] = dtab + (2 * a + d) * kMaxRhs;
    g.lam[a] = reinterpret_cast<const double* const*>(dtab + (6 + a) * kMaxRhs);
    g.coef[a] = reinterpret_cast<const double* const*>(dtab + (10 + a) * kMaxRhs);
  }
  g.lamxy = reinterpret_cast<const double* const*>(dtab + 9 * kMaxRhs);
  g.rhs_plan = owner.data();
  return helm::solve_impl(p0, f, u, total, sig.data(), ws, stream, info, false, &g);
}

// The solve sequence shared by helm_solve and helm_solve_noalloc.  noalloc: the call must not
// allocate anything, so the two paths that create objects on demand are refused (EINVAL):
// adaptive refinement (its norms are read back through pinned host memory and a per-thread
// event) and stage timing (its events are created lazily).
helm_status helm::solve_impl(helm_plan* p, const double* f, double* u, int nrhs, const double* sigma_per_rhs,
                             void* ws, void* stream, helm_info* info, bool noalloc, const GroupTabs* grp) {
  if (!p || !f || !u || nrhs < 1 || nrhs > kMaxRhs) return HELM_EINVAL;
  if (p->refined() && f == u) return HELM_EINVAL;
  if (noalloc && (p->prof.on || (p->refined() && p->opts.ir_tol != 0.0))) return HELM_EINVAL;
  size_t total = 0, off_a = 0, off_b = 0, off_n = 0, off_m = 0, off_c = 0;
  workspace_layout(p, nrhs, &total, &off_a, &off_b, &off_n, &off_m, &off_c);
  if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0) return HELM_EINVAL;
  double sig[kMaxRhs];
  for (int r = 0; r < nrhs; ++r) {
    sig[r] = sigma_per_rhs ? sigma_per_rhs[r] : p->sigma;
    if (!std::isfinite(sig[r])) return HELM_EINVAL;
    const helm_plan* pr_r = grp ? grp->rhs_plan[r] : p;  // the plan that owns RHS r
    if (p->cyl && sig[r] < 0.0) return HELM_EINVAL;
    if (!p->cyl && sig[r] != pr_r->sigma && has_zero_denominator(pr_r, sig[r])) return HELM_ESINGULAR;
  }
  DeviceGuard dg(p->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const Prec pr = p->prec();
  // All-Neumann Laplace RHS (sigma = 0, projection mode): the divide sets the null-mode
  // coefficient to exactly zero, and the volume-weighted mean of u is that coefficient times a
  // constant, so an FP64 solve leaves a mean at the rounding level (~1e-16 |u|) and needs no
  // pass of its own.  A low-precision first solve leaks a constant at its own precision that
  // no refinement sweep can see (H 1 = 0); it is removed at the end with an FP64
  // volume-weighted mean.
  unsigned long long null_mask = 0;
  for (int r = 0; r < nrhs; ++r) {
    const helm_plan* pr_r = grp ? grp->rhs_plan[r] : p;
    if (pr_r->all_neumann && p->opts.null_mode == HELM_NULL_PROJECT && sig[r] == 0.0) null_mask |= 1ull << r;
  }
  // a grouped low-precision solve has no per-plan volume tables for the final projection
  if (grp && null_mask && pr != P_F64) return HELM_EINVAL;
  auto project_null = [&]() -> hipError_t {
    if (!null_mask) return hipSuccess;
    double vs = 1.0;
    for (int d = 0; d < 3; ++d) {
      double t = 0.0;
      for (double v : p->ax[d]->host.vol) t += v;
      vs *= t;
    }
    return timed(p, HELM_STAGE_OTHER, st, [&] {
      return remove_mean(u, p->ax[0]->vol, p->ax[1]->vol, p->ax[2]->vol, p->m[0], p->m[1], p->m[2], nrhs, 1.0 / vs,
                         null_mask, reinterpret_cast<double*>(w + off_m), st);
    });
  };
  if (info) {
    info->sweeps = 1;
    info->last_correction = 0.0;
    info->converged = 1;
    info->iterations = 0;
    info->residual = 0.0;
  }
  hipError_t e = hipSuccess;
  if (pr == P_F64) {
    double* W = reinterpret_cast<double*>(w + off_a);
    const DevAxis& X = *p->ax[0];
    const DevAxis& Y = *p->ax[1];
    const DevAxis& Z = *p->ax[2];
    const long long nx = p->m[0], ny = p->m[1], nz = p->m[2];
    if (!p->thomas()) {  // TPF, and HELM_FFT (TPF with fast transforms on uniform axes)
      // f -> W -> u -> W -> u -> W -> u  (u may alias f: f is consumed by the first product)
      e = tpf_products(p, P_F64, f, W, u, u, EPI_STORE, nrhs, sig, nullptr, 0, st, false, false, nullptr, grp);
    } else {
      if (grp) return HELM_EINVAL;
      EpiArgs ep;
      ep.nx = static_cast<int>(nx);
      ThomasArgs ta;
      ta.kdiag = Z.kdiag;
      ta.koff = Z.koff;
      ta.vol = Z.vol;
      ta.lamx = X.lam;
      ta.lamy = Y.lam;
      ta.gdiag = p->cyl ? Z.gdiag : nullptr;  // eq. 44: the theta eigenvalue enters through 1 / r^2
      ta.nx = static_cast<int>(nx);
      ta.ny = static_cast<int>(ny);
      ta.nz = static_cast<int>(nz);
      ta.nrhs = nrhs;
      bool null_line = false;
      for (int r = 0; r < nrhs; ++r) {
        ta.sigma[r] = sig[r];
        null_line = null_line || (p->all_neumann && sig[r] == 0.0);
      }
      // The singular (0,0) line exists only for RHS with sigma = 0 on an all-Neumann plan;
      // when every RHS has it, Thomas skips the line and the eigen path solves it.
      bool all_null = true;
      for (int r = 0; r < nrhs; ++r) all_null = all_null && p->all_neumann && sig[r] == 0.0;
      if (null_line && !all_null) return HELM_EINVAL;  // mixed shifts on a singular plan: not supported
      ta.skip_null = all_null ? 1 : 0;
      if (e == hipSuccess)
        e = timed(p, HELM_STAGE_X_FWD, st, [&] {
          return mode_right(P_F64, X.sw[0][0], nx, f, P_F64, W, P_F64, nrhs * ny * nz, EPI_STORE, ep, st);
        });
      if (e == hipSuccess)
        e = timed(p, HELM_STAGE_Y_FWD, st, [&] {
          return mode_left(P_F64, Y.sw[0][0], ny, W, P_F64, u, P_F64, nrhs * nz, nx, EPI_STORE, ep, st);
        });
      if (e == hipSuccess) e = timed(p, HELM_STAGE_THOMAS, st, [&] { return thomas_z(u, ta, w + off_b, st); });
      if (e == hipSuccess && all_null)
        e = timed(p, HELM_STAGE_NULL_LINE, st, [&] {
          // W is free here (Y_FWD consumed it, Y_INV rewrites it): it holds the line's modes
          return null_line_z(u, Z.E, Z.Einv, Z.lam, ta.nx, ta.ny, ta.nz, nrhs,
                             p->opts.null_mode == HELM_NULL_PAPER_EQ28, W, st);
        });
      if (e == hipSuccess)
        e = timed(p, HELM_STAGE_Y_INV, st, [&] {
          return mode_left(P_F64, Y.sw[0][1], ny, u, P_F64, W, P_F64, nrhs * nz, nx, EPI_STORE, ep, st);
        });
      if (e == hipSuccess)
        e = timed(p, HELM_STAGE_X_INV, st, [&] {
          return mode_right(P_F64, X.sw[0][1], nx, W, P_F64, u, P_F64, nrhs * ny * nz, EPI_STORE, ep, st);
        });
    }
    return from_hip(e);
  }

  // Low-precision products, optionally refined.
  void* L1 = w + off_a;
  void* L2 = w + off_b;
  unsigned long long* norms = reinterpret_cast<unsigned long long*>(w + off_n);
  if (grp && pr != P_BF16X3) return HELM_EINVAL;
  const StencilArgs sa = stencil_args(p, nrhs, sig, grp);
  const Prec store = pr == P_BF16X3 ? P_F32 : pr;  // storage type of the low-precision fields
  // Sweep 0: L1 = low(f) (the residual of u = 0), u = M^{-1} L1.  Its norms are not read: the
  // first correction is measured against u itself.
  // Split-BF16 with refinement sweeps to follow keeps the first solve in FP32 (L3): the first
  // residual and update then read 4 bytes of it per point instead of 8.
  float* U0 = nullptr;
  if (pr == P_BF16X3 && p->refined() && p->opts.max_sweeps > 1) U0 = reinterpret_cast<float*>(w + off_c);
  if (pr == P_BF16X3) {  // the first product reads f in FP64 directly
    if (e == hipSuccess)
      e = tpf_products(p, pr, f, L2, L1, U0 ? static_cast<void*>(U0) : static_cast<void*>(u), EPI_ACCUM, nrhs, sig,
                       norms, 1, st, true, U0 != nullptr, nullptr, grp);
  } else {
    if (e == hipSuccess)
      e = timed(p, HELM_STAGE_CONVERT, st, [&] { return stencil(2, nullptr, f, L1, store, sa, st); });
    if (e == hipSuccess) e = tpf_products(p, pr, L1, L2, L1, u, EPI_ACCUM, nrhs, sig, norms, 1, st);
  }
  if (e != hipSuccess) return from_hip(e);
  if (!p->refined()) return from_hip(project_null());
  // ir_tol = 0: a fixed sweep count with no norm read back (nothing allocated, nothing waited on)
  const bool fixed = p->opts.ir_tol == 0.0;
  std::optional<PinnedNorms> hn;  // pinned host copy of the norm stripes, from a process-wide pool
  if (!fixed) {
    hn.emplace();
    if (!hn->p) return HELM_ENOMEM;
  }
  int sweeps = 1;
  double last = 0.0, prev = 1.0;  // the first solve's "correction" is u itself
  bool conv = false;
  while (sweeps < p->opts.max_sweeps) {
    const float* u0 = sweeps == 1 ? U0 : nullptr;  // the iterate is still the FP32 first solve
    StencilArgs sz = sa;  // the residual also clears this sweep's norm stripes
    sz.zero = norms;
    sz.nzero = 2 * nrhs * kNormStripes;
    if (e == hipSuccess)
      e = timed(p, HELM_STAGE_RESIDUAL, st, [&] {
        return u0 ? stencil_u32(1, u0, f, L1, store, sz, st) : stencil(1, u, f, L1, store, sz, st);
      });
    if (e == hipSuccess)
      e = tpf_products(p, pr, L1, L2, L1, u, EPI_ACCUM, nrhs, sig, norms, 0, st, false, false, u0, grp);
    if (e == hipSuccess && !fixed)
      e = hipMemcpyAsync(hn->p, norms, 2 * nrhs * kNormStripes * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && !fixed) e = helm::wait_stream(st);
    if (e != hipSuccess) return from_hip(e);
    ++sweeps;
    if (fixed) continue;
    last = 0.0;
    bool finite = true;
    for (int r = 0; r < nrhs; ++r) {
      // the stripes hold non-negative FP64 bit patterns (NaN as the largest): integer max
      unsigned long long bd = 0, bu = 0;
      for (int q = 0; q < kNormStripes; ++q) {
        bd = std::max(bd, hn->p[(2 * r) * kNormStripes + q]);
        bu = std::max(bu, hn->p[(2 * r + 1) * kNormStripes + q]);
      }
      double dm, um;
      std::memcpy(&dm, &bd, 8);
      std::memcpy(&um, &bu, 8);
      if (!std::isfinite(dm) || !std::isfinite(um)) finite = false;
      const double rel = um > 0.0 ? dm / um : (dm > 0.0 ? INFINITY : 0.0);
      last = std::max(last, rel);
    }
    if (!finite) {
      if (info) {
        info->sweeps = sweeps;
        info->last_correction = last;
        info->converged = 0;
      }
      return HELM_ENONFINITE;
    }
    // Stop when the correction is below tolerance, or when the observed contraction
    // rho = last / prev predicts the next correction (the remaining error) below it.
    const double rho = last / prev;
    if (last <= p->opts.ir_tol || (rho < 0.5 && rho * last <= p->opts.ir_tol)) {
      conv = true;
      break;
    }
    prev = last;
  }
  if (info) {
    info->sweeps = sweeps;
    info->last_correction = fixed ? -1.0 : last;
    info->converged = fixed ? -1 : (conv ? 1 : 0);
  }
  if ((e = project_null()) != hipSuccess) return from_hip(e);
  return (conv || fixed) ? HELM_OK : HELM_ENOTCONVERGED;
}

extern "C" helm_status helm_pressure_setup(const helm_grid* grid, const helm_opts* opts, helm_plan** out) {
  if (!grid) return HELM_EINVAL;
  helm_grid g = *grid;
  for (int d = 0; d < 3; ++d) g.loc[d] = HELM_CELL;
  helm_bc bc;
  for (int d = 0; d < 3; ++d) bc.lo[d] = bc.hi[d] = HELM_NEUMANN;
  return helm_setup(&g, &bc, 0.0, opts, out);
}

extern "C" helm_status helm_pressure_solve(helm_plan* p, const double* f, double* pr, int nrhs, void* ws, void* stream,
                                           helm_info* info) {
  if (!p || !p->all_neumann || p->sigma != 0.0) return HELM_EINVAL;
  return helm_solve(p, f, pr, nrhs, nullptr, ws, stream, info);
}

extern "C" helm_status helm_fast_axes(const helm_plan* p, int* mask) {
  if (!p || !mask) return HELM_EINVAL;
  *mask = 0;
  if (p->opts.method == HELM_FFT && !p->cyl)
    for (int d = 0; d < 3; ++d)
      if (p->ax[d]->fft_ok) *mask |= 1 << d;
  return HELM_OK;
}

extern "C" helm_status helm_profile_enable(helm_plan* p, int enable) {
  if (!p) return HELM_EINVAL;
  p->prof.on = enable != 0;
  p->prof.clear();
  return HELM_OK;
}

extern "C" helm_status helm_profile_stages(helm_plan* p, unsigned stage_mask) {
  if (!p || (stage_mask & ((1u << HELM_NSTAGES) - 1u)) == 0) return HELM_EINVAL;
  p->prof.mask = stage_mask;
  p->prof.clear();
  return HELM_OK;
}

extern "C" helm_status helm_profile_read(helm_plan* p, double* ms, int* launches) {
  if (!p || !ms || !launches) return HELM_EINVAL;
  for (int i = 0; i < HELM_NSTAGES; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (const auto& r : p->prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return HELM_EDEVICE;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return HELM_EDEVICE;
    ms[r.stage] += t;
    launches[r.stage] += 1;
  }
  p->prof.clear();
  return HELM_OK;
}
