// Continuous-batching solve server (include/helm.h, "Serving").
//
// The time-stepping use of the solver (Section 5, eqs. 37-40) issues a stream of Helmholtz
// and Poisson solves of different shifts and right-hand-side counts, whose cost does not
// depend on the time step (Section 1).  The server keeps the eigenbases resident, admits
// queued requests by free slot and device-workspace budget, and runs each admitted request on
// its slot's stream from the slot's worker thread, so requests overlap on the GPU and new
// ones are admitted while others are in flight.  Queued requests on the plan of a request being
// admitted ride along with it: one multi-RHS solve with every request's shifts (the velocity
// components of a time step share their grids), their f and u staged contiguously.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/helm.h"
#include "alloc.hpp"
#include "kernels.hpp"
#include "solve_impl.hpp"

namespace {

// ---------------------------------------------------------------- admission policy
// Size classes (unknowns x right-hand sides of one solve).  Each kernel of a solve of
// kBigPoints or more fills the GPU by itself, so two such solves at once only share it while
// every kernel of a smaller concurrent request queues behind theirs: at most one big solve
// runs at a time, and smaller requests may pass a big one that waits for it.  Requests ride
// along with an admitted one while the solve stays within kBatchPoints: batching pays for
// small grids, whose launches are short, and past that only lengthens the kernels that every
// concurrent request waits behind.
constexpr long long kBigPoints = 1LL << 23;
constexpr long long kBatchPoints = 1LL << 25;

struct Pending {
  double t_submit;
  size_t foot;
  bool big;  // at least kBigPoints
};

// Index (in the arrival-ordered queue) of the next request to admit, or -1.  A request is
// admissible when its workspace fits and it is not big while a big solve runs.  The head is
// admitted when admissible; otherwise a later admissible request may pass it only while the
// head has waited less than max_bypass (after that, capacity is reserved for the head).
// fits(foot): whether a workspace of `foot` bytes can be had now.
template <typename Q, typename Fits>
int pick_next(const Q& queue, int free_slots, Fits&& fits, double now, double max_bypass, bool big_running) {
  if (free_slots <= 0 || queue.empty()) return -1;
  auto ok = [&](size_t i) {
    const Pending p = queue[i];
    return fits(p.foot) && !(big_running && p.big);
  };
  if (ok(0)) return 0;
  if (now - queue.front().t_submit >= max_bypass) return -1;
  for (size_t i = 1; i < queue.size(); ++i)
    if (ok(i)) return static_cast<int>(i);
  return -1;
}

// First-fit allocator of byte ranges (256-byte granules) inside the server's workspace arena:
// the arena is the whole HBM budget, allocated once at creation, so the memory the server holds
// is the budget itself and no device allocation happens while requests are in flight.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  // Largest contiguous free range.
  size_t largest() const {
    size_t m = 0;
    for (auto& b : free_) m = std::max(m, b.second);
    return m;
  }
  // Offset of a range of `bytes` (rounded up to 256), or SIZE_MAX if none is free.
  size_t take(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        return off;
      }
    return SIZE_MAX;
  }
  void give(size_t off, size_t bytes) {
    bytes = round(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  static size_t round(size_t b) { return (b + 255) / 256 * 256; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

// Plans are shared between the resident map and the requests that use them; the last owner
// destroys the plan (an evicted plan stays alive until its queued and running requests finish).
// Every solve a worker enqueues is waited for before its requests are released, so a plan
// whose last reference goes has no work in flight: it is freed without helm_destroy's
// device-wide synchronization, which would stall the submitting thread (evictions happen in
// submit) behind every running solve.
using PlanRef = std::shared_ptr<helm_plan>;
inline PlanRef adopt(helm_plan* p) { return PlanRef(p, [](helm_plan* q) { helm::release_plan(q); }); }

// Resident plans kept per server (least recently used evicted beyond this).  A plan owns no
// large memory of its own: its 1D eigenbases are shared through the per-axis cache and a split-
// BF16 plan's lambda_x + lambda_y table through the per-axis-pair cache, both alive while some
// plan uses them.  The bound is large so that the axes of a workload stay referenced (an
// evicted axis is rebuilt by the extended-precision eigensolver) and small enough that the
// pair tables stay within a few hundred MB.
constexpr size_t kMaxResidentPlans = 2048;

struct Request {
  long long id = 0;
  PlanRef plan;
  std::vector<double> sigma;
  int nrhs = 0;
  long long npts = 0;  // unknowns per right-hand side
  const double* f = nullptr;
  double* u = nullptr;
  double t_submit = 0.0, t_admit = 0.0;
  size_t foot = 0;  // bytes charged: the solve's workspace (+ staging when others ride along)
  long long batch_points = 0;  // unknowns x right-hand sides of its solve, riders included
  bool big = false;            // that solve is of the big class (set at admission)
  long long points() const { return npts * nrhs; }
  size_t off = 0;   // arena offset of the workspace (set at admission)
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream: f is written
  std::vector<std::unique_ptr<Request>> riders;  // same-plan requests solved with this one
};

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace of a batch of `total` right-hand sides led by plan p: a grouped solve's (the plan's
// own layout plus the per-RHS operand table), which also serves a batch on p alone; 0 when the
// size cannot be had.
inline size_t batch_ws(helm_plan* p, int total) {
  size_t ws = 0;
  if (helm_group_workspace_size(&p, 1, &total, &ws) != HELM_OK) return 0;
  return ws;
}
// Footprint of one batch solve with staging for f and u, or 0 when the size cannot be had.
inline size_t batch_foot(helm_plan* p, int total, long long npts) {
  const size_t ws = batch_ws(p, total);
  if (ws == 0) return 0;
  return align256(ws) + 2 * static_cast<size_t>(total) * static_cast<size_t>(npts) * sizeof(double);
}

struct Slot {
  std::thread worker;
  hipStream_t stream = nullptr;
  void* ws = nullptr;            // the running job's workspace (inside the arena)
  std::unique_ptr<Request> job;  // assigned request (null when idle)
  std::condition_variable cv;
};

}  // namespace

struct helm_server {
  size_t budget = 0;
  double max_bypass = 0.0;
  helm_opts opts{};
  int device = 0;
  helm::DevAlloc alloc;     // allocator of the arena (opts.alloc, else hipMalloc)
  unsigned char* arena_mem = nullptr;
  size_t arena_bytes = 0;
  Arena arena;              // guarded by mu
  std::vector<hipEvent_t> events;  // idle submit events, guarded by mu
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<std::unique_ptr<Slot>> slots;
  std::deque<helm_request_record> done;
  size_t used = 0;
  long long submitted = 0, completed = 0;
  bool stop = false;
  std::mutex plan_mu;
  struct Resident {
    PlanRef plan;
    unsigned long long last_use = 0;
  };
  std::map<std::string, Resident> plans;
  unsigned long long use_clock = 0;
  long long plan_hits = 0, plan_misses = 0;  // guarded by plan_mu
  double setup_seconds = 0.0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Admit as many queued requests as the policy allows (called with mu held).
  void admit_locked() {
    for (;;) {
      int free_slots = 0;
      for (auto& s : slots)
        if (!s->job) ++free_slots;
      struct View {
        const std::deque<std::unique_ptr<Request>>& q;
        bool empty() const { return q.empty(); }
        size_t size() const { return q.size(); }
        Pending operator[](size_t i) const { return {q[i]->t_submit, q[i]->foot, q[i]->points() >= kBigPoints}; }
        Pending front() const { return (*this)[0]; }
      } view{queue};
      bool big_running = false;
      for (auto& s : slots) big_running = big_running || (s->job && s->job->big);
      const size_t largest = arena.largest();
      auto fits = [&](size_t foot) { return Arena::round(foot) <= largest; };
      const int i = pick_next(view, free_slots, fits, now(), max_bypass, big_running);
      if (i < 0) return;
      std::unique_ptr<Request> r = std::move(queue[i]);
      queue.erase(queue.begin() + i);
      r->t_admit = now();
      // beside a running big solve the batch stays below the big class
      add_riders(r.get(), largest, big_running ? kBigPoints - 1 : kBatchPoints);
      r->big = r->batch_points >= kBigPoints;
      r->off = arena.take(r->foot);  // fits: checked against the largest free range above
      used += r->foot;
      for (auto& s : slots)
        if (!s->job) {
          s->ws = arena_mem + r->off;
          s->job = std::move(r);
          s->cv.notify_one();
          break;
        }
    }
  }

  // Pull queued requests into r's solve while the right-hand sides fit one solve (64), the
  // solve's unknowns stay within max_points (r alone may exceed it) and the grown footprint
  // fits the budget: requests on r's plan, and requests on other grids of r's shape that a
  // grouped solve can take (each multiplied by its own plan's eigenbases).  Riders pass
  // requests queued before them only while the head of the queue has waited less than
  // max_bypass (or is itself the rider).
  void add_riders(Request* r, size_t largest, long long max_points) {
    int total = r->nrhs;
    r->batch_points = r->points();
    const double t = now();
    for (size_t j = 0; j < queue.size();) {
      Request& q = *queue[j];
      const bool head_ok = j == 0 || t - queue.front()->t_submit < max_bypass;
      const bool joins = q.plan == r->plan || helm::plans_groupable(r->plan.get(), q.plan.get());
      if (!joins || total + q.nrhs > 64 || !head_ok || (total + q.nrhs) * r->npts > max_points) {
        ++j;
        continue;
      }
      const size_t grown = batch_foot(r->plan.get(), total + q.nrhs, r->npts);
      if (grown == 0 || Arena::round(grown) > largest) break;
      r->foot = grown;
      total += q.nrhs;
      r->batch_points = total * r->npts;
      queue[j]->t_admit = t;
      r->riders.push_back(std::move(queue[j]));
      queue.erase(queue.begin() + j);
    }
  }

  // One request alone, or a batch as one multi-RHS (one plan) or grouped (several grids of one
  // shape) solve through staging buffers after the solve's workspace; a batch the solver
  // refuses (e.g. mixed singular and regular shifts on an all-Neumann plan) is solved request
  // by request.  Returns a status per request.
  std::vector<helm_status> run(Request& r, Slot& s, helm_info& info) {
    std::vector<Request*> reqs{&r};
    for (auto& q : r.riders) reqs.push_back(q.get());
    std::vector<helm_status> out(reqs.size(), HELM_OK);
    // every request's right-hand side is complete once its submitter's stream reaches the
    // point recorded at submit
    for (Request* q : reqs)
      if (q->ready && hipStreamWaitEvent(s.stream, q->ready, 0) != hipSuccess) {
        std::fill(out.begin(), out.end(), HELM_EDEVICE);
        return out;
      }
    // the stream is waited for whatever the status: a failed solve may have enqueued work
    auto one = [&](Request& q) -> helm_status {
      helm_status st = helm_solve(q.plan.get(), q.f, q.u, q.nrhs, q.sigma.data(), s.ws, s.stream, &info);
      const hipError_t we = helm::wait_stream(s.stream);
      if (st == HELM_OK && we != hipSuccess) st = HELM_EDEVICE;
      return st;
    };
    if (reqs.size() == 1) {
      out[0] = one(r);
      return out;
    }
    int total = 0;
    std::vector<double> sig;
    std::vector<helm_plan*> plans;
    std::vector<int> counts;
    bool one_plan = true;
    for (Request* q : reqs) {
      total += q->nrhs;
      sig.insert(sig.end(), q->sigma.begin(), q->sigma.end());
      plans.push_back(q->plan.get());
      counts.push_back(q->nrhs);
      one_plan = one_plan && q->plan == r.plan;
    }
    const size_t ws = batch_ws(r.plan.get(), total);
    helm_status st = ws ? HELM_OK : HELM_EINVAL;
    double* F = reinterpret_cast<double*>(static_cast<char*>(s.ws) + align256(ws));
    double* U = F + static_cast<size_t>(total) * r.npts;
    const size_t per = static_cast<size_t>(r.npts) * sizeof(double);
    size_t o = 0;
    for (Request* q : reqs) {
      if (st == HELM_OK && hipMemcpyAsync(F + o * r.npts, q->f, q->nrhs * per, hipMemcpyDeviceToDevice, s.stream) !=
                               hipSuccess)
        st = HELM_EDEVICE;
      o += q->nrhs;
    }
    if (st == HELM_OK)
      st = one_plan ? helm_solve(r.plan.get(), F, U, total, sig.data(), s.ws, s.stream, &info)
                    : helm_solve_group(plans.data(), static_cast<int>(plans.size()), counts.data(), F, U, sig.data(),
                                       s.ws, s.stream, &info);
    if (st == HELM_EINVAL) {
      for (size_t i = 0; i < reqs.size(); ++i) out[i] = one(*reqs[i]);
      return out;
    }
    if (st == HELM_OK || st == HELM_ENOTCONVERGED) {
      o = 0;
      for (Request* q : reqs) {
        if (hipMemcpyAsync(q->u, U + o * r.npts, q->nrhs * per, hipMemcpyDeviceToDevice, s.stream) != hipSuccess)
          st = HELM_EDEVICE;
        o += q->nrhs;
      }
    }
    const hipError_t we = helm::wait_stream(s.stream);
    if ((st == HELM_OK || st == HELM_ENOTCONVERGED) && we != hipSuccess) st = HELM_EDEVICE;
    std::fill(out.begin(), out.end(), st);
    return out;
  }

  void work(int k) {
    (void)hipSetDevice(device);
    Slot& s = *slots[k];
    for (;;) {
      std::unique_ptr<Request>* jp = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        s.cv.wait(lk, [&] { return stop || s.job != nullptr; });
        if (!s.job) return;  // stop requested and idle
        jp = &s.job;
      }
      Request& r = **jp;
      helm_info info{};
      std::vector<helm_status> sts = run(r, s, info);
      const double t_done = now();
      std::vector<helm_request_record> recs;
      for (size_t i = 0; i < sts.size(); ++i) {
        const Request& q = i == 0 ? r : *r.riders[i - 1];
        helm_request_record rec{};
        rec.id = q.id;
        rec.status = sts[i];
        rec.sweeps = info.sweeps;
        rec.last_correction = info.last_correction;
        rec.t_submit = q.t_submit;
        rec.t_admit = q.t_admit;
        rec.t_done = t_done;
        rec.footprint = r.foot;
        rec.slot = k;
        rec.batch = static_cast<int>(sts.size());
        recs.push_back(rec);
      }
      std::unique_ptr<Request> finished;
      {
        std::lock_guard<std::mutex> lk(mu);
        used -= r.foot;
        arena.give(r.off, r.foot);
        if (r.ready) events.push_back(r.ready);
        for (auto& q : r.riders)
          if (q->ready) events.push_back(q->ready);
        s.ws = nullptr;
        finished = std::move(s.job);
        for (auto& rec : recs) done.push_back(rec);
        completed += static_cast<long long>(recs.size());
        admit_locked();
      }
      // released outside the lock: dropping the last reference to an evicted plan frees its
      // device memory, possibly through the caller's allocator callback
      finished.reset();
      cv_done.notify_all();
    }
  }
};

namespace {
std::string plan_key(const helm_grid* g, const helm_bc* bc) {
  std::string k;
  for (int d = 0; d < 3; ++d) {
    k.append(reinterpret_cast<const char*>(&g->n[d]), sizeof(int));
    k.append(reinterpret_cast<const char*>(g->faces[d]), sizeof(double) * (g->n[d] + 1));
    k.push_back(static_cast<char>(g->loc[d]));
    k.push_back(static_cast<char>(bc->lo[d]));
    k.push_back(static_cast<char>(bc->hi[d]));
  }
  return k;
}
}  // namespace

extern "C" helm_status helm_server_create(size_t hbm_budget_bytes, int slots, double max_bypass_ms,
                                          const helm_opts* opts, helm_server** out) {
  if (!out || slots < 1 || slots > 16 || hbm_budget_bytes == 0 || !(max_bypass_ms >= 0.0)) return HELM_EINVAL;
  *out = nullptr;
  std::unique_ptr<helm_server> s(new (std::nothrow) helm_server());
  if (!s) return HELM_ENOMEM;
  s->budget = hbm_budget_bytes;
  s->max_bypass = max_bypass_ms * 1e-3;
  helm_default_opts(&s->opts);
  if (opts) s->opts = *opts;
  if (hipGetDevice(&s->device) != hipSuccess) return HELM_EDEVICE;
  s->t0 = std::chrono::steady_clock::now();
  s->alloc = helm::DevAlloc::from(s->opts);
  if (!s->alloc.valid()) return HELM_EINVAL;
  // the whole budget as one arena: the server holds exactly this much device memory
  s->arena_bytes = Arena::round(hbm_budget_bytes);
  void* mem = nullptr;
  if (s->alloc.get(&mem, s->arena_bytes) != hipSuccess) return HELM_ENOMEM;
  s->arena_mem = static_cast<unsigned char*>(mem);
  s->arena.reset(s->arena_bytes);
  // from here a failure releases what was made through helm_server_destroy, which takes a
  // partly built server (no worker, no stream yet)
  helm_server* raw = s.release();
  for (int k = 0; k < slots; ++k) {
    auto sl = std::make_unique<Slot>();
    const bool ok = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess;
    raw->slots.push_back(std::move(sl));
    if (!ok) {
      helm_server_destroy(raw);
      return HELM_EDEVICE;
    }
  }
  try {
    for (int k = 0; k < slots; ++k) raw->slots[k]->worker = std::thread([raw, k] { raw->work(k); });
  } catch (const std::system_error&) {
    helm_server_destroy(raw);
    return HELM_ENOMEM;
  }
  *out = raw;
  return HELM_OK;
}

extern "C" helm_status helm_server_submit(helm_server* s, const helm_grid* grid, const helm_bc* bc, const double* sigma,
                                          int nrhs, const double* f, double* u, long long id, void* stream) {
  if (!s || !grid || !bc || !sigma || !f || !u || nrhs < 1 || nrhs > 64) return HELM_EINVAL;
  const double t_submit = s->now();
  PlanRef plan;
  {
    std::lock_guard<std::mutex> lk(s->plan_mu);
    const std::string key = plan_key(grid, bc);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {
      plan = it->second.plan;
      it->second.last_use = ++s->use_clock;
      ++s->plan_hits;
    } else {
      const auto t_setup = std::chrono::steady_clock::now();
      helm_plan* raw = nullptr;
      const helm_status st = helm_setup(grid, bc, 0.0, &s->opts, &raw);
      if (st != HELM_OK) return st;
      plan = adopt(raw);
      if (s->plans.size() >= kMaxResidentPlans) {
        auto lru = s->plans.begin();
        for (auto jt = s->plans.begin(); jt != s->plans.end(); ++jt)
          if (jt->second.last_use < lru->second.last_use) lru = jt;
        s->plans.erase(lru);
      }
      s->plans[key] = helm_server::Resident{plan, ++s->use_clock};
      ++s->plan_misses;
      s->setup_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_setup).count();
    }
  }
  auto r = std::make_unique<Request>();
  r->id = id;
  r->plan = plan;
  r->sigma.assign(sigma, sigma + nrhs);
  r->nrhs = nrhs;
  r->npts = 1;
  for (int d = 0; d < 3; ++d) r->npts *= grid->loc[d] == HELM_FACE ? grid->n[d] - 1 : grid->n[d];
  r->f = f;
  r->u = u;
  r->t_submit = t_submit;
  helm_status st = helm_workspace_size(plan.get(), nrhs, &r->foot);
  if (st != HELM_OK) return st;
  if (Arena::round(r->foot) > s->arena_bytes) return HELM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->events.empty()) {
      r->ready = s->events.back();
      s->events.pop_back();
    }
  }
  if (!r->ready && hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) return HELM_EDEVICE;
  if (hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->events.push_back(r->ready);
    return HELM_EDEVICE;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->queue.push_back(std::move(r));
    ++s->submitted;
    s->admit_locked();
  }
  return HELM_OK;
}

extern "C" helm_status helm_server_poll(helm_server* s, helm_request_record* out, int max, int* n, int wait_ms) {
  if (!s || !n || (max > 0 && !out)) return HELM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return HELM_OK;
}

extern "C" helm_status helm_server_stats(helm_server* s, helm_server_stats_t* out) {
  if (!s || !out) return HELM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->submitted;
    out->completed = s->completed;
  }
  std::lock_guard<std::mutex> lk(s->plan_mu);
  out->plan_hits = s->plan_hits;
  out->plan_misses = s->plan_misses;
  out->setup_seconds = s->setup_seconds;
  return HELM_OK;
}

extern "C" helm_status helm_server_drain(helm_server* s) {
  if (!s) return HELM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
  return HELM_OK;
}

extern "C" double helm_server_now(const helm_server* s) { return s ? s->now() : 0.0; }

extern "C" void helm_server_destroy(helm_server* s) {
  if (!s) return;
  helm_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  for (auto& sl : s->slots) sl->cv.notify_all();
  for (auto& sl : s->slots) {
    if (sl->worker.joinable()) sl->worker.join();
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
  }
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  s->alloc.put(s->arena_mem, s->arena_bytes);
  s->plans.clear();
  delete s;
}

// ---------------------------------------------------------------- virtual-clock simulation
extern "C" helm_status helm_sched_simulate(int n, const double* arrival, const double* service, const size_t* foot,
                                           const int* big, int slots, size_t budget, double max_bypass_ms,
                                           double* admit, double* done) {
  if (n < 0 || slots < 1 || (n > 0 && (!arrival || !service || !foot || !admit || !done))) return HELM_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (foot[i] > budget || !(service[i] >= 0.0)) return HELM_EINVAL;
    if (i > 0 && arrival[i] < arrival[i - 1]) return HELM_EINVAL;
  }
  const double max_bypass = max_bypass_ms * 1e-3;
  struct Q {
    std::deque<int> idx;
    const double* arr;
    const size_t* ft;
    const int* bg;
    bool empty() const { return idx.empty(); }
    size_t size() const { return idx.size(); }
    Pending operator[](size_t i) const { return {arr[idx[i]], ft[idx[i]], bg && bg[idx[i]] != 0}; }
    Pending front() const { return (*this)[0]; }
  } q{{}, arrival, foot, big};
  std::vector<std::pair<double, int>> running;  // (finish time, request)
  size_t used = 0;
  int next = 0, finished = 0;
  double now = 0.0;
  while (finished < n) {
    // next event: an arrival or the earliest completion
    double t_arr = next < n ? arrival[next] : 1e300;
    double t_fin = 1e300;
    for (auto& r : running) t_fin = std::min(t_fin, r.first);
    now = std::min(t_arr, t_fin);
    // completions at `now`
    for (size_t i = 0; i < running.size();) {
      if (running[i].first <= now) {
        used -= foot[running[i].second];
        ++finished;
        running.erase(running.begin() + i);
      } else {
        ++i;
      }
    }
    while (next < n && arrival[next] <= now) q.idx.push_back(next++);
    for (;;) {
      auto fits = [&](size_t f) { return used + f <= budget; };
      bool big_running = false;
      for (auto& r : running) big_running = big_running || (big && big[r.second] != 0);
      const int i = pick_next(q, slots - static_cast<int>(running.size()), fits, now, max_bypass, big_running);
      if (i < 0) break;
      const int r = q.idx[i];
      q.idx.erase(q.idx.begin() + i);
      admit[r] = now;
      done[r] = now + service[r];
      used += foot[r];
      running.push_back({done[r], r});
    }
  }
  return HELM_OK;
}
