// Continuous-batching reconstruction server.
//
// A scheduler thread owns one HBM arena (allocated once; requests are carved
// out of it first-fit, so admission is an allocation against the budget) and
// a pool of streams.  Every tick it admits the request at the head of the
// queue together with every queued request of the same kind (grid,
// supersampling, precision, preconditioning), as many as fit, as one cohort:
// a batched solve whose every pass is one launch for all its requests, each
// with its own mask, prior, box and CG scalars.  Cohorts of every kind run
// concurrently on their own streams and advance without being waited on:
// when a cohort's last enqueued work has completed (an event), the scheduler
// reads its CG states (copied back with that work) and enqueues reliable
// updates, the next chunk of iterations, or, for a request whose solve has
// stopped, its final transform and the copy of its result.  Gridding
// transients go back to the arena as soon as the data vectors are built.
// Krylov state never leaves the device.  A request's arithmetic touches only
// its own slices and reduces in a fixed order whatever the cohort, so its
// result is bitwise the same alone and in any mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "checks.h"
#include "internal.h"
#include "solver.h"

using namespace wf;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

void* arena_alloc(size_t bytes, void* user) { return static_cast<Arena*>(user)->get(bytes); }
void arena_free(void* p, void* user) { static_cast<Arena*>(user)->put(p); }

constexpr int MAX_COHORT = 16;   // requests per batched solve
// With more than one stream, the last free stream takes only requests of
// grids up to SMALL_N^3: a small request then never waits behind large
// solves (tens of ms against hundreds), and large ones still have the other
// streams, which are enough to keep HBM busy.
constexpr int SMALL_N = 128;

enum JobPhase : int { J_QUEUED = 0, J_ACTIVE, J_DONE, J_FAILED };
enum SlotPhase : int { S_RUNNING = 0, S_COPYING, S_DONE, S_FAILED };

struct Job {
  uint64_t ticket = 0;
  // request (host copies, kept until its cohort has read them)
  int n = 0;
  double box = 0.0;
  std::vector<double> w, p, xyz;
  int64_t n_gal = 0;
  int scheme = 0, ss = 1;
  wf_solve_opts opts{};
  bool mixed = true;
  bool split = false;
  // written by the scheduler thread before `phase` becomes J_DONE / J_FAILED,
  // read by the API threads after
  std::atomic<int> phase{J_QUEUED};
  std::atomic<bool> cancelled{false};
  std::vector<double> result;
  wf_solve_info info{};
  Clock::time_point t_submit, t_start, t_done;
  std::string err;
};

// Requests of equal grid, supersampling, precision and preconditioning
// admitted together: one solve with a batch dimension (every pass one launch
// for all of them, blockIdx.y the request), each request with its own mask,
// prior tables, box and scalars.  A request finishes, and its result is
// copied out, as soon as its own solve has stopped.
struct Cohort {
  int n = 0, ss = 1, k = 0, chunk = 16;
  bool mixed = true, split = false;
  std::vector<std::shared_ptr<Job>> jobs;
  std::vector<int> slot;          // SlotPhase per request
  OperatorData od;                // per-request tables (strides rhs_*)
  SolveWork sw;
  // gridding transients, released once the data vectors are built
  DepositWork dw;
  DevBuf xyz_d, nobs, staging, parts;
  bool dep_pending = false;
  DevBuf scal;                    // per request: sumw, nbar; then flag words
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr, dep_ev = nullptr;
  bool in_flight = false;         // work enqueued since the last completed ev
  void release_transients() {
    dw.grid.release();
    dw.fine_spec.release();
    dw.spec_y.release();
    dw.spec_c.release();
    dw.tw_fine.release();
    dw.tw_fine_n = 0;
    xyz_d.release();
    nobs.release();
    staging.release();
    parts.release();
  }
  void release_all() {
    release_transients();
    for (DevBuf* b : {&od.w64, &od.w32, &od.tw64, &od.tw32, &od.lam64, &od.xlam64, &od.xlam32,
                      &od.fac64, &od.fac32, &sw.b64, &sw.x64, &sw.r64, &sw.p64, &sw.q64,
                      &sw.spec64, &sw.x32, &sw.r32, &sw.p32, &sw.q32, &sw.spec32, &sw.bh64,
                      &sw.u64, &sw.state, &sw.partials, &scal})
      b->release();
  }
};

}  // namespace

struct wf_server {
  int device = 0;
  Allocator outer;       // caller's allocator (arena storage)
  Arena arena;
  Allocator al;          // arena allocator handed to the cohorts
  void* arena_mem = nullptr;
  int max_active = 1;    // batched solves in flight (one stream each)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Job>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<hipStream_t> streams;   // idle streams
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string err;
  // scheduler thread only
  std::vector<std::unique_ptr<Cohort>> cohorts;
  int active_jobs = 0;
  // statistics (under mu)
  std::vector<double> latencies;
  int64_t failed = 0;
  int64_t n_cohorts = 0;
  int largest_cohort = 0;
  bool have_first = false;
  Clock::time_point first_submit, last_done;

  void run();
  bool admit_some();
  Status build(Cohort& c, const std::vector<std::shared_ptr<Job>>& js);
  Status setup(Cohort& c);
  void advance(Cohort& c);
  void finish_job(Cohort& c, int i, bool ok);
  void fail_job(const std::shared_ptr<Job>& j, wf_status code, const std::string& why);
};

namespace {

Status validate_request(const wf_request& r) {
  wf_status code = WF_OK;
  if (const char* e = request_error(r, &code)) return fail(code, e);
  return {};
}

// Device bytes of a cohort of one request: its tables, its solve state and
// the gridding transients (the sizes build() allocates), plus granule rounding.
size_t job_footprint(int n, int ss, bool mixed, bool split, int64_t n_gal) {
  Grid g;
  g.set(n, 1.0);
  size_t f = footprint_bytes(n, ss, mixed ? WF_MIXED : WF_FP64, 1, split);
  f += (size_t)n_gal * 24 + (size_t)std::max<int64_t>(g.m, g.lamlen) * 8 + 4096 * 8 + 64 * 1024;
  f += 48 * 256;
  return f;
}

bool same_key(const Job& a, const Job& b) {
  return a.n == b.n && a.ss == b.ss && a.mixed == b.mixed && a.split == b.split;
}

}  // namespace

void wf_server::fail_job(const std::shared_ptr<Job>& j, wf_status code, const std::string& why) {
  j->info = wf_solve_info{};
  j->info.status = code;
  j->err = why;
  std::lock_guard<std::mutex> g(mu);
  failed += 1;
  j->phase.store(J_FAILED);
}

// Allocates the cohort's buffers for requests js (all-or-nothing).
Status wf_server::build(Cohort& c, const std::vector<std::shared_ptr<Job>>& js) {
  const Job& j0 = *js[0];
  c.k = (int)js.size();
  c.n = j0.n;
  c.ss = j0.ss;
  c.mixed = j0.mixed;
  c.split = j0.split;
  c.jobs = js;
  c.slot.assign(c.k, S_RUNNING);
  c.chunk = 1 << 30;
  int64_t max_gal = 1;
  for (const auto& j : js) {
    c.chunk = std::min(c.chunk, j->opts.check_every > 0 ? j->opts.check_every : 16);
    max_gal = std::max(max_gal, j->n_gal);
  }
  OperatorData& od = c.od;
  od.g.set(c.n, j0.box);
  const Grid& g = od.g;
  const int k = c.k;
  const int64_t facl = split_fac_elems(c.n);
  od.rhs_w = g.m;
  od.rhs_lam = g.lamlen;
  od.rhs_xlam = g.xlamlen;
  od.rhs_fac = c.split ? facl : 0;
  WF_TRY(od.w64.ensure(al, (size_t)k * g.m * 8));
  WF_TRY(od.w32.ensure(al, (size_t)k * g.m * 4));
  WF_TRY(od.lam64.ensure(al, (size_t)k * g.lamlen * 8));
  WF_TRY(od.xlam64.ensure(al, (size_t)k * g.xlamlen * 8));
  WF_TRY(od.xlam32.ensure(al, (size_t)k * g.xlamlen * 4));
  if (c.split) {
    WF_TRY(od.fac64.ensure(al, (size_t)k * facl * 8));
    WF_TRY(od.fac32.ensure(al, (size_t)k * facl * 4));
  }
  WF_TRY(c.sw.ensure(al, g, k, !c.mixed, c.mixed, c.split));
  WF_TRY(c.scal.ensure(al, (size_t)(2 * k + 8) * 8));
  WF_TRY(c.xyz_d.ensure(al, (size_t)max_gal * 24));
  WF_TRY(c.nobs.ensure(al, (size_t)g.m * 8));
  WF_TRY(c.staging.ensure(al, (size_t)std::max<int64_t>(g.m, g.lamlen) * 8));
  WF_TRY(c.parts.ensure(al, 4096 * 8));
  const int nf = c.ss * g.n;
  WF_TRY(c.dw.grid.ensure(al, (size_t)nf * nf * nf * 8));
  if (c.ss == 2) {
    const int h = g.n / 2;
    WF_TRY(c.dw.fine_spec.ensure(al, (size_t)nf * nf * h * 16));
    WF_TRY(c.dw.spec_y.ensure(al, (size_t)nf * g.n * h * 16));
    WF_TRY(c.dw.spec_c.ensure(al, (size_t)g.spec_total * 16));
    WF_TRY(make_twiddles(al, nf, c.dw.tw_fine, nullptr, c.stream));
    c.dw.tw_fine_n = nf;
  }
  WF_TRY(make_twiddles(al, g.n, od.tw64, &od.tw32, c.stream));
  return {};
}

// Enqueues the set-up of every request (tables, gridding, data vector, solver
// state), the start of the batched solve and its first chunk.
Status wf_server::setup(Cohort& c) {
  hipStream_t s = c.stream;
  OperatorData& od = c.od;
  const Grid& g = od.g;
  const int k = c.k;
  double* scal = c.scal.as<double>();
  int* flags = reinterpret_cast<int*>(scal + 2 * k);
  uint32_t* ticket = reinterpret_cast<uint32_t*>(scal + 2 * k + 2);
  WF_HIP(launch_fill_f64(scal, 2 * k + 8, s));
  const int64_t facl = split_fac_elems(c.n);
  for (int i = 0; i < k; ++i) {
    Job& j = *c.jobs[i];
    double* sumw = scal + 2 * i;
    double* nbar = scal + 2 * i + 1;
    WF_HIP(hipMemcpyAsync(c.staging.p, j.w.data(), (size_t)g.m * 8, hipMemcpyHostToDevice, s));
    WF_HIP(launch_mask(c.staging.as<double>(), od.w64.as<double>() + i * g.m,
                       od.w32.as<float>() + i * g.m, g.m, flags, c.parts.as<double>(), ticket,
                       sumw, s));
    WF_HIP(hipMemcpyAsync(c.staging.p, j.p.data(), (size_t)g.lamlen * 8, hipMemcpyHostToDevice, s));
    const double h = j.box / g.n;
    double* lam = od.lam64.as<double>() + i * g.lamlen;
    WF_HIP(launch_lambda(c.staging.as<double>(), g.lamlen, h * h * h, 1.0 / (double)g.m, lam,
                         flags + 1, s));
    WF_HIP(launch_xlam_rows(g.n, lam, od.xlam64.as<double>() + i * g.xlamlen,
                            od.xlam32.as<float>() + i * g.xlamlen, s));
    if (c.split)
      WF_HIP(launch_split_fac(g.n, lam, (double)g.m, od.fac64.as<double>() + i * facl,
                              od.fac32.as<float>() + i * facl, s));
    if (j.n_gal > 0)
      WF_HIP(hipMemcpyAsync(c.xyz_d.p, j.xyz.data(), (size_t)j.n_gal * 24, hipMemcpyHostToDevice,
                            s));
    OperatorData view;
    view.make_view(od, i, j.box);
    WF_TRY(run_deposit(al, view, c.dw, c.xyz_d.as<double>(), j.n_gal, j.scheme, c.ss,
                       c.nobs.as<double>(), s));
    WF_HIP(launch_data_vector(c.nobs.as<double>(), od.w64.as<double>() + i * g.m, sumw,
                              (double)j.n_gal, nbar, c.sw.b64.as<double>() + i * g.m, g.m, s));
    const wf_solve_opts& o = j.opts;
    WF_HIP(launch_state_init(c.sw.state.as<CgState>() + i, nbar, o.tol, o.max_iter,
                             o.inner_tol > 0 ? o.inner_tol : 0.1, o.max_outer,
                             effective_err_tol(o), 1, s));
  }
  od.fac_ready = c.split;
  WF_HIP(hipEventRecord(c.dep_ev, s));
  c.dep_pending = true;
  WF_TRY(solve_start(od, c.sw, k, c.mixed, s));
  WF_TRY(solve_chunk(od, c.sw, k, c.mixed, c.chunk, s));
  WF_HIP(hipMemcpyAsync(c.sw.st_host, c.sw.state.p, sizeof(CgState) * k, hipMemcpyDeviceToHost, s));
  WF_HIP(hipEventRecord(c.ev, s));
  c.in_flight = true;
  return {};
}

// Admits the first queued request (when only the reserved stream is free, the
// first small one) together with every queued request of the same kind (up
// to MAX_COHORT), as many of them as fit in the arena; returns true if a
// cohort was started or a request retired.
bool wf_server::admit_some() {
  std::vector<std::shared_ptr<Job>> cand;
  std::shared_ptr<Job> head;
  hipStream_t st = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    while (!queue.empty() && queue.front()->cancelled.load()) {
      auto j = queue.front();
      queue.pop_front();
      j->info = wf_solve_info{};
      j->info.status = WF_ESTATE;
      j->err = "cancelled";
      failed += 1;
      j->phase.store(J_FAILED);
    }
    if (queue.empty() || streams.empty()) return false;
    const bool reserved = max_active > 1 && streams.size() == 1;
    for (const auto& j : queue) {
      if (j->cancelled.load() || (reserved && j->n > SMALL_N)) continue;
      head = j;
      break;
    }
    if (!head) return false;  // only large requests wait: the last stream is kept
    for (const auto& j : queue) {
      if ((int)cand.size() >= MAX_COHORT) break;
      if (!j->cancelled.load() && same_key(*head, *j)) cand.push_back(j);
    }
    st = streams.back();
  }
  std::unique_ptr<Cohort> c;
  Status why;
  for (int k = (int)cand.size(); k >= 1; --k) {
    c = std::make_unique<Cohort>();
    c->stream = st;
    std::vector<std::shared_ptr<Job>> js(cand.begin(), cand.begin() + k);
    why = build(*c, js);
    if (why.ok()) break;
    // nothing of this attempt is queued on the stream any more: give it back
    (void)hipStreamSynchronize(st);
    c->release_all();
    c.reset();
  }
  if (!c) {
    bool idle;
    {
      std::lock_guard<std::mutex> g(mu);
      idle = cohorts.empty();
    }
    if (!idle) return false;  // wait for memory to come back
    // nothing will free memory: the head request cannot run
    {
      std::lock_guard<std::mutex> g(mu);
      queue.erase(std::find(queue.begin(), queue.end(), head));
    }
    fail_job(head, why.code, why.msg);
    return true;
  }
  {
    std::lock_guard<std::mutex> g(mu);
    for (const auto& j : c->jobs) queue.erase(std::find(queue.begin(), queue.end(), j));
    streams.pop_back();
    active_jobs += c->k;
    n_cohorts += 1;
    largest_cohort = std::max(largest_cohort, c->k);
  }
  if (hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->dep_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    for (auto& j : c->jobs) fail_job(j, WF_EDEVICE, "event creation failed");
    c->slot.assign(c->k, S_FAILED);
    cohorts.push_back(std::move(c));
    return true;
  }
  const auto now = Clock::now();
  for (auto& j : c->jobs) {
    j->t_start = now;
    j->phase.store(J_ACTIVE);
  }
  Status e = setup(*c);
  if (!e.ok()) {
    for (auto& j : c->jobs) fail_job(j, e.code, e.msg);
    c->slot.assign(c->k, S_FAILED);
  }
  cohorts.push_back(std::move(c));
  return true;
}

void wf_server::finish_job(Cohort& c, int i, bool ok) {
  auto& j = c.jobs[i];
  if (!ok) return;
  j->t_done = Clock::now();
  const Grid& g = c.od.g;
  solve_infos(c.sw.st_host + i, 1, c.mixed, c.split, g, ms_between(j->t_start, j->t_done),
              &j->info);
  j->info.latency_ms = ms_between(j->t_submit, j->t_done);
  std::lock_guard<std::mutex> lk(mu);
  latencies.push_back(ms_between(j->t_submit, j->t_done));
  last_done = j->t_done;
  j->phase.store(J_DONE);
}

// One scheduling step of a cohort whose last enqueued work has completed.
void wf_server::advance(Cohort& c) {
  hipStream_t s = c.stream;
  if (c.dep_pending && hipEventQuery(c.dep_ev) == hipSuccess) {
    c.release_transients();
    c.dep_pending = false;
  }
  if (!c.in_flight) return;
  const hipError_t q = hipEventQuery(c.ev);
  if (q == hipErrorNotReady) return;
  c.in_flight = false;
  auto fail_all = [&](wf_status code, const std::string& why) {
    for (int i = 0; i < c.k; ++i)
      if (c.slot[i] == S_RUNNING || c.slot[i] == S_COPYING) {
        c.slot[i] = S_FAILED;
        fail_job(c.jobs[i], code, why);
      }
  };
  if (q != hipSuccess) {
    fail_all(WF_EDEVICE, hipGetErrorString(q));
    return;
  }
  auto step = [&]() -> Status {
    bool running = false, update = false, enq = false;
    for (int i = 0; i < c.k; ++i) {
      if (c.slot[i] == S_COPYING) {  // its result copy has completed
        c.slot[i] = S_DONE;
        finish_job(c, i, true);
        continue;
      }
      if (c.slot[i] != S_RUNNING) continue;
      auto& j = c.jobs[i];
      const CgState& st = c.sw.st_host[i];
      if (j->cancelled.load()) {
        WF_HIP(launch_state_stop(c.sw.state.as<CgState>() + i, s));
        c.slot[i] = S_FAILED;
        fail_job(j, WF_ESTATE, "cancelled");
        enq = true;
      } else if (c.mixed && st.status == CG_UPDATE) {
        update = running = true;
      } else if (st.done) {
        // this request has stopped: s = C y and its true residual (views of
        // its slot), then its result to the host
        SolveWork v;
        v.make_view(c.sw, c.od.g, i);
        OperatorData ov;
        ov.make_view(c.od, i, j->box);
        WF_TRY(solve_finish(ov, v, 1, c.mixed, s));
        j->result.resize(c.od.g.m);
        WF_HIP(hipMemcpyAsync(j->result.data(), v.x64.p, (size_t)c.od.g.m * 8,
                              hipMemcpyDeviceToHost, s));
        c.slot[i] = S_COPYING;
        enq = true;
      } else {
        running = true;
      }
    }
    if (update) WF_TRY(solve_update(c.od, c.sw, c.k, s));
    if (running) WF_TRY(solve_chunk(c.od, c.sw, c.k, c.mixed, c.chunk, s));
    if (enq || running) {
      WF_HIP(hipMemcpyAsync(c.sw.st_host, c.sw.state.p, sizeof(CgState) * c.k,
                            hipMemcpyDeviceToHost, s));
      WF_HIP(hipEventRecord(c.ev, s));
      c.in_flight = true;
    }
    return {};
  };
  Status e = step();
  if (!e.ok()) fail_all(e.code, e.msg);
}

void wf_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    bool progressed = false;
    while (admit_some()) progressed = true;
    for (auto& c : cohorts) {
      const bool was = c->in_flight;
      advance(*c);
      progressed = progressed || (was && !c->in_flight);
    }
    // retire cohorts whose requests have all finished
    for (size_t i = 0; i < cohorts.size();) {
      Cohort& c = *cohorts[i];
      bool all = !c.in_flight;
      for (int t = 0; t < c.k && all; ++t) all = c.slot[t] == S_DONE || c.slot[t] == S_FAILED;
      if (!all) {
        ++i;
        continue;
      }
      (void)hipStreamSynchronize(c.stream);
      c.release_all();
      if (c.ev) (void)hipEventDestroy(c.ev);
      if (c.dep_ev) (void)hipEventDestroy(c.dep_ev);
      for (auto& j : c.jobs) {
        std::vector<double>().swap(j->w);
        std::vector<double>().swap(j->p);
        std::vector<double>().swap(j->xyz);
      }
      {
        std::lock_guard<std::mutex> g(mu);
        streams.push_back(c.stream);
        active_jobs -= c.k;
      }
      cohorts.erase(cohorts.begin() + i);
      progressed = true;
    }
    std::unique_lock<std::mutex> lk(mu);
    if (stop && cohorts.empty() && queue.empty()) break;
    if (!progressed) {
      if (cohorts.empty() && (queue.empty() || stop))
        cv.wait_for(lk, std::chrono::milliseconds(50));
      else
        cv.wait_for(lk, std::chrono::microseconds(30));
    }
  }
}

extern "C" {

wf_status wf_server_create(wf_server** out, int device, size_t budget, int32_t max_active,
                           wf_alloc_fn alloc, wf_free_fn free_fn, void* user) {
  if (!out || max_active <= 0 || budget < (1u << 20)) return WF_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return WF_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return WF_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return WF_EDEVICE;
  auto* s = new (std::nothrow) wf_server();
  if (!s) return WF_ENOMEM;
  s->device = device;
  s->outer.alloc = alloc;
  s->outer.free_fn = free_fn;
  s->outer.user = user;
  s->outer.device = device;
  s->arena_mem = s->outer.get(budget);
  if (!s->arena_mem) {
    delete s;
    return WF_ENOMEM;
  }
  s->arena.init(s->arena_mem, budget);
  s->al.alloc = arena_alloc;
  s->al.free_fn = arena_free;
  s->al.user = &s->arena;
  s->al.device = device;
  s->max_active = max_active;
  for (int i = 0; i < max_active; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      s->outer.put(s->arena_mem);
      delete s;
      return WF_EDEVICE;
    }
    s->streams.push_back(st);
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return WF_OK;
}

wf_status wf_server_submit(wf_server* s, const wf_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return WF_EINVAL;
  Status v = validate_request(*r);
  if (!v.ok()) {
    std::lock_guard<std::mutex> g(s->mu);
    s->err = v.msg;
    return v.code;
  }
  const bool mixed = r->opts.precision == WF_MIXED;
  const bool split = r->opts.precond == WF_PRECOND_PRIOR;
  const size_t need = job_footprint(r->n, r->supersample, mixed, split, r->n_gal);
  if (need > s->arena.size) {
    std::lock_guard<std::mutex> g(s->mu);
    s->err = "request needs " + std::to_string(need) + " bytes, the budget is " +
             std::to_string(s->arena.size);
    return WF_ENOMEM;
  }
  auto j = std::make_shared<Job>();
  Grid g;
  g.set(r->n, r->box_mpc);
  j->n = r->n;
  j->box = r->box_mpc;
  j->w.assign(r->w, r->w + g.m);
  j->p.assign(r->p_by_m2, r->p_by_m2 + g.lamlen);
  if (r->n_gal > 0) j->xyz.assign(r->xyz, r->xyz + 3 * r->n_gal);
  j->n_gal = r->n_gal;
  j->scheme = r->scheme;
  j->ss = r->supersample;
  j->opts = r->opts;
  j->mixed = mixed;
  j->split = split;
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return WF_ESTATE;
    j->ticket = s->next_ticket++;
    if (!s->have_first) {
      s->have_first = true;
      s->first_submit = j->t_submit;
    }
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv.notify_all();
  return WF_OK;
}

wf_status wf_server_poll(wf_server* s, uint64_t ticket, int32_t* done, wf_solve_info* info) {
  if (!s || !done) return WF_EINVAL;
  std::shared_ptr<Job> j;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) {
      s->err = "unknown ticket";
      return WF_EINVAL;
    }
    j = it->second;
  }
  const int ph = j->phase.load();
  const bool fin = ph == J_DONE || ph == J_FAILED;
  *done = fin ? 1 : 0;
  if (fin && info) *info = j->info;
  return WF_OK;
}

wf_status wf_server_fetch(wf_server* s, uint64_t ticket, double* out) {
  if (!s || !out) return WF_EINVAL;
  std::shared_ptr<Job> j;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) {
      s->err = "unknown ticket";
      return WF_EINVAL;
    }
    j = it->second;
    const int ph = j->phase.load();
    if (ph != J_DONE && ph != J_FAILED) {
      s->err = "request not finished";
      return WF_ESTATE;
    }
    s->jobs.erase(it);
    if (ph == J_FAILED) {
      s->err = j->err;
      return j->info.status != WF_OK ? (wf_status)j->info.status : WF_EDEVICE;
    }
  }
  std::memcpy(out, j->result.data(), j->result.size() * 8);
  return (wf_status)j->info.status;
}

wf_status wf_server_cancel(wf_server* s, uint64_t ticket) {
  if (!s) return WF_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return WF_EINVAL;
  it->second->cancelled.store(true);
  return WF_OK;
}

wf_status wf_server_stats_get(wf_server* s, wf_server_stats* out) {
  if (!s || !out) return WF_EINVAL;
  *out = wf_server_stats{};
  {
    std::lock_guard<std::mutex> g(s->mu);
    out->completed = (int64_t)s->latencies.size();
    out->failed = s->failed;
    out->cohorts = s->n_cohorts;
    out->largest_cohort = s->largest_cohort;
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    if (!l.empty()) {
      auto pct = [&](double q) {
        size_t k = (size_t)std::ceil(q * l.size());
        if (k < 1) k = 1;
        return l[std::min(k, l.size()) - 1];
      };
      out->p50_ms = pct(0.50);
      out->p99_ms = pct(0.99);
      const double span = ms_between(s->first_submit, s->last_done) * 1e-3;
      out->solves_per_s = span > 0 ? l.size() / span : 0.0;
    }
  }
  {
    std::lock_guard<std::mutex> g(s->arena.mu);
    out->peak_bytes = s->arena.peak;
  }
  return WF_OK;
}

const char* wf_server_last_error(const wf_server* s) { return s ? s->err.c_str() : "null server"; }

wf_status wf_server_destroy(wf_server* s) {
  if (!s) return WF_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (auto& kv : s->jobs) kv.second->cancelled.store(true);
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  s->outer.put(s->arena_mem);
  delete s;
  return WF_OK;
}

}  // extern "C"
