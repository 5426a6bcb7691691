// Continuous-batching reconstruction server.
//
// A scheduler thread owns one HBM arena (allocated once; requests are carved
// out of it first-fit, so admission is an allocation against the budget) and
// one stream per active request.  Every tick it admits queued requests while
// their buffers fit and fewer than max_active run, and advances each active
// request without waiting on it: when the request's last enqueued chunk has
// completed (an event), it reads the request's CG state (copied back with
// the chunk) and enqueues the next chunk of iterations, a reliable update, or
// the result copy.  Krylov state never leaves the device; requests of every
// grid size run concurrently on their own streams.  A request's arithmetic
// touches only its own buffers and reduces in a fixed order, so its result
// is bitwise the same alone and in any mix.
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

#include "internal.h"
#include "solver.h"

using namespace wf;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit arena over one device allocation; 256-byte granules.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::mutex mu;
  std::map<size_t, size_t> free_;   // offset -> bytes
  std::map<size_t, size_t> used_;   // offset -> bytes
  size_t in_use = 0, peak = 0;

  void init(void* p, size_t n) {
    base = static_cast<char*>(p);
    size = n & ~size_t(255);
    free_.clear();
    used_.clear();
    free_[0] = size;
    in_use = peak = 0;
  }
  void* get(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    std::lock_guard<std::mutex> g(mu);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, left = it->second - bytes;
      free_.erase(it);
      if (left) free_[off + bytes] = left;
      used_[off] = bytes;
      in_use += bytes;
      peak = std::max(peak, in_use);
      return base + off;
    }
    return nullptr;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    const size_t off = static_cast<char*>(p) - base;
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    in_use -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }
};

void* arena_alloc(size_t bytes, void* user) { return static_cast<Arena*>(user)->get(bytes); }
void arena_free(void* p, void* user) { static_cast<Arena*>(user)->put(p); }

enum Phase { QUEUED, RUNNING, FINAL_RES, COPYING, DONE, FAILED };

struct Job {
  uint64_t ticket = 0;
  // request (host copies)
  int n = 0;
  double box = 0.0;
  std::vector<double> w, p, xyz;
  int64_t n_gal = 0;
  int scheme = 0, ss = 1;
  wf_solve_opts opts{};
  bool mixed = true;
  bool split = false;
  // device side
  OperatorData od;
  DepositWork dw;
  SolveWork sw;
  DevBuf xyz_d, nobs, scal, staging;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  Phase phase = QUEUED;
  bool cancelled = false;
  // results
  std::vector<double> result;
  wf_solve_info info{};
  Clock::time_point t_submit, t_start, t_done;
  std::string err;
};

}  // namespace

struct wf_server {
  int device = 0;
  Allocator outer;       // caller's allocator (arena storage)
  Arena arena;
  Allocator al;          // arena allocator handed to the jobs
  void* arena_mem = nullptr;
  int max_active = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Job>> queue;
  std::vector<std::shared_ptr<Job>> active;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<hipStream_t> streams;   // idle streams
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string err;
  // statistics
  std::vector<double> latencies;
  int64_t failed = 0;
  bool have_first = false;
  Clock::time_point first_submit, last_done;
  std::atomic<size_t> peak{0};

  void run();
  bool admit(const std::shared_ptr<Job>& j, Status& why);
  bool advance(const std::shared_ptr<Job>& j);
  void retire(const std::shared_ptr<Job>& j, bool ok);
};

namespace {

Status validate_request(const wf_request& r) {
  Grid g;
  int m = r.n;
  if (r.n < 8 || r.n > 512) return fail(WF_EINVAL, "n out of range");
  while (m % 2 == 0) m /= 2;
  if (m != 1 && m != 3) return fail(WF_EINVAL, "n must be 2^a 3^b (b <= 1)");
  if (!(r.box_mpc > 0.0) || !std::isfinite(r.box_mpc)) return fail(WF_EINVAL, "bad box");
  if (!r.w || !r.p_by_m2 || (r.n_gal > 0 && !r.xyz) || r.n_gal < 0)
    return fail(WF_EINVAL, "null request array");
  if (r.n_gal >= (int64_t(1) << 24)) return fail(WF_EOVERFLOW, "n_gal must be < 2^24");
  if (r.scheme < WF_NGP || r.scheme > WF_TSC || (r.supersample != 1 && r.supersample != 2))
    return fail(WF_EINVAL, "bad scheme or supersample");
  WF_TRY(validate_opts(r.opts));
  g.set(r.n, r.box_mpc);
  double sw = 0.0;
  for (int64_t i = 0; i < g.m; ++i) {
    const double v = r.w[i];
    if (!(v >= 0.0 && v <= 1.0)) return fail(WF_EINVAL, "mask values must be in [0, 1]");
    sw += v;
  }
  if (!(sw > 0.0)) return fail(WF_EINVAL, "mask is zero everywhere");
  for (int64_t j = 1; j < g.lamlen; ++j)
    if (!(r.p_by_m2[j] > 0.0) || !std::isfinite(r.p_by_m2[j]))
      return fail(WF_EINVAL, "P(k) must be finite and > 0");
  for (int64_t i = 0; i < 3 * r.n_gal; ++i)
    if (!(r.xyz[i] >= 0.0 && r.xyz[i] < r.box_mpc))
      return fail(WF_EINVAL, "galaxy coordinates must satisfy 0 <= x < L");
  return {};
}

size_t job_footprint(int n, int ss, bool mixed, bool split, int64_t n_gal) {
  Grid g;
  g.set(n, 1.0);
  size_t f = footprint_bytes(n, ss, mixed ? WF_MIXED : WF_FP64, 1, split);
  f += (size_t)n_gal * 24 + (size_t)g.m * 8 /* staging */ + (size_t)g.lamlen * 8 + 64 * 1024;
  f += 48 * 256;  // granule rounding of every buffer
  return f;
}

}  // namespace

bool wf_server::admit(const std::shared_ptr<Job>& j, Status& why) {
  // allocate everything up front; on failure give it all back and wait
  j->od.g.set(j->n, j->box);
  const Grid& g = j->od.g;
  auto attempt = [&]() -> Status {
    hipStream_t s = j->stream;
    WF_TRY(j->od.w64.ensure(al, (size_t)g.m * 8));
    WF_TRY(j->od.w32.ensure(al, (size_t)g.m * 4));
    WF_TRY(j->od.lam64.ensure(al, (size_t)g.lamlen * 8));
    WF_TRY(alloc_xlam(al, j->od));
    if (j->split) WF_TRY(alloc_split_fac(al, j->od));
    WF_TRY(j->xyz_d.ensure(al, (size_t)std::max<int64_t>(j->n_gal, 1) * 24));
    WF_TRY(j->nobs.ensure(al, (size_t)g.m * 8));
    WF_TRY(j->scal.ensure(al, 64 * 8));
    WF_TRY(j->staging.ensure(al, std::max<size_t>((size_t)g.lamlen * 8, 4096 * 8)));
    WF_TRY(j->sw.ensure(al, g, 1, !j->mixed, j->mixed, j->split));
    const int nf = j->ss * g.n;
    WF_TRY(j->dw.grid.ensure(al, (size_t)nf * nf * nf * 8));
    if (j->ss == 2) {
      const int h = g.n / 2;
      WF_TRY(j->dw.fine_spec.ensure(al, (size_t)nf * nf * h * 16));
      WF_TRY(j->dw.spec_y.ensure(al, (size_t)nf * g.n * h * 16));
      WF_TRY(j->dw.spec_c.ensure(al, (size_t)g.spec_total * 16));
      WF_TRY(make_twiddles(al, nf, j->dw.tw_fine, nullptr, s));
      j->dw.tw_fine_n = nf;
    }
    WF_TRY(make_twiddles(al, g.n, j->od.tw64, &j->od.tw32, s));
    return {};
  };
  Status st = attempt();
  if (!st.ok()) {
    why = st;
    return false;
  }
  peak.store(std::max(peak.load(), arena.peak));
  // enqueue the whole set-up and the first chunk on the request's stream
  auto enqueue = [&]() -> Status {
    hipStream_t s = j->stream;
    double* scal = j->scal.as<double>();
    WF_HIP(launch_fill_f64(scal, 64, s));
    // mask (staged through n_obs), prior table, galaxies
    WF_HIP(hipMemcpyAsync(j->nobs.p, j->w.data(), (size_t)g.m * 8, hipMemcpyHostToDevice, s));
    WF_HIP(launch_mask(j->nobs.as<double>(), j->od.w64.as<double>(), j->od.w32.as<float>(), g.m,
                       reinterpret_cast<int*>(scal + 16), j->staging.as<double>(),
                       reinterpret_cast<uint32_t*>(scal + 8), scal, s));
    WF_HIP(hipMemcpyAsync(j->staging.p, j->p.data(), (size_t)g.lamlen * 8, hipMemcpyHostToDevice, s));
    const double h = g.box / g.n;
    WF_HIP(launch_lambda(j->staging.as<double>(), g.lamlen, h * h * h, 1.0 / (double)g.m,
                         j->od.lam64.as<double>(), reinterpret_cast<int*>(scal + 17), s));
    WF_TRY(build_xlam(j->od, s));
    if (j->split) WF_TRY(build_split_fac(j->od, s));
    if (j->n_gal > 0)
      WF_HIP(hipMemcpyAsync(j->xyz_d.p, j->xyz.data(), (size_t)j->n_gal * 24, hipMemcpyHostToDevice, s));
    // gridding, data vector, solver state
    WF_TRY(run_deposit(al, j->od, j->dw, j->xyz_d.as<double>(), j->n_gal, j->scheme, j->ss,
                       j->nobs.as<double>(), s));
    WF_HIP(launch_data_vector(j->nobs.as<double>(), j->od.w64.as<double>(), scal, (double)j->n_gal,
                              scal + 1, j->sw.b64.as<double>(), g.m, s));
    const wf_solve_opts& o = j->opts;
    WF_HIP(launch_state_init(j->sw.state.as<CgState>(), scal + 1, o.tol, o.max_iter,
                             o.inner_tol > 0 ? o.inner_tol : 0.1, o.max_outer, 1, s));
    WF_TRY(solve_start(j->od, j->sw, 1, j->mixed, s));
    const int chunk = o.check_every > 0 ? o.check_every : 16;
    WF_TRY(solve_chunk(j->od, j->sw, 1, j->mixed, chunk, s));
    WF_HIP(hipMemcpyAsync(j->sw.st_host, j->sw.state.p, sizeof(CgState), hipMemcpyDeviceToHost, s));
    WF_HIP(hipEventRecord(j->ev, s));
    return {};
  };
  j->t_start = Clock::now();
  Status e = enqueue();
  if (!e.ok()) {
    j->err = e.msg;
    j->info.status = e.code;
    j->phase = FAILED;
    return true;
  }
  j->phase = RUNNING;
  return true;
}

bool wf_server::advance(const std::shared_ptr<Job>& j) {
  if (j->phase == DONE || j->phase == FAILED) return false;
  const hipError_t q = hipEventQuery(j->ev);
  if (q == hipErrorNotReady) return false;
  if (q != hipSuccess) {
    j->err = hipGetErrorString(q);
    j->info.status = WF_EDEVICE;
    j->phase = FAILED;
    return true;
  }
  hipStream_t s = j->stream;
  const int chunk = j->opts.check_every > 0 ? j->opts.check_every : 16;
  auto step = [&]() -> Status {
    if (j->phase == RUNNING) {
      const CgState& c = j->sw.st_host[0];
      if (j->cancelled) {
        j->phase = FAILED;
        j->info.status = WF_ESTATE;
        j->err = "cancelled";
        return {};
      }
      if (j->mixed && c.status == CG_UPDATE) {
        WF_TRY(solve_update(j->od, j->sw, 1, s));
        WF_TRY(solve_chunk(j->od, j->sw, 1, true, chunk, s));
      } else if (c.done) {
        if (!j->mixed || j->split) {
          WF_TRY(solve_finish(j->od, j->sw, 1, j->mixed, s));
          j->phase = FINAL_RES;
        } else {
          j->result.resize(j->od.g.m);
          WF_HIP(hipMemcpyAsync(j->result.data(), j->sw.x64.p, (size_t)j->od.g.m * 8,
                                hipMemcpyDeviceToHost, s));
          j->phase = COPYING;
        }
      } else {
        WF_TRY(solve_chunk(j->od, j->sw, 1, j->mixed, chunk, s));
      }
    } else if (j->phase == FINAL_RES) {
      j->result.resize(j->od.g.m);
      WF_HIP(hipMemcpyAsync(j->result.data(), j->sw.x64.p, (size_t)j->od.g.m * 8,
                            hipMemcpyDeviceToHost, s));
      j->phase = COPYING;
    } else if (j->phase == COPYING) {
      j->t_done = Clock::now();
      solve_infos(j->sw.st_host, 1, j->mixed, j->split, j->od.g, ms_between(j->t_start, j->t_done),
                  &j->info);
      j->phase = DONE;
      return {};
    }
    WF_HIP(hipMemcpyAsync(j->sw.st_host, j->sw.state.p, sizeof(CgState), hipMemcpyDeviceToHost, s));
    WF_HIP(hipEventRecord(j->ev, s));
    return {};
  };
  Status e = step();
  if (!e.ok()) {
    j->err = e.msg;
    j->info.status = e.code;
    j->phase = FAILED;
  }
  return true;
}

void wf_server::retire(const std::shared_ptr<Job>& j, bool ok) {
  (void)hipStreamSynchronize(j->stream);
  // give the request's device memory back to the arena
  j->od.w64.release();
  j->od.w32.release();
  j->od.lam64.release();
  j->od.xlam64.release();
  j->od.xlam32.release();
  j->od.fac64.release();
  j->od.fac32.release();
  j->sw.bh64.release();
  j->sw.u64.release();
  j->od.tw64.release();
  j->od.tw32.release();
  j->dw.grid.release();
  j->dw.fine_spec.release();
  j->dw.spec_y.release();
  j->dw.spec_c.release();
  j->dw.tw_fine.release();
  j->xyz_d.release();
  j->nobs.release();
  j->scal.release();
  j->staging.release();
  for (DevBuf* b : {&j->sw.b64, &j->sw.x64, &j->sw.r64, &j->sw.p64, &j->sw.q64, &j->sw.spec64,
                    &j->sw.x32, &j->sw.r32, &j->sw.p32, &j->sw.q32, &j->sw.spec32, &j->sw.bh64, &j->sw.u64, &j->sw.state,
                    &j->sw.partials})
    b->release();
  std::vector<double>().swap(j->w);
  std::vector<double>().swap(j->p);
  std::vector<double>().swap(j->xyz);
  std::lock_guard<std::mutex> g(mu);
  streams.push_back(j->stream);
  j->stream = nullptr;
  if (ok && !j->cancelled) {
    latencies.push_back(ms_between(j->t_submit, j->t_done));
    last_done = j->t_done;
  } else {
    failed += 1;
  }
}

void wf_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    bool progressed = false;
    // admission: FIFO, while buffers fit and slots are free
    for (;;) {
      std::shared_ptr<Job> j;
      {
        std::lock_guard<std::mutex> g(mu);
        if (queue.empty() || (int)active.size() >= max_active || streams.empty()) break;
        j = queue.front();
        if (j->cancelled) {
          queue.pop_front();
          j->phase = FAILED;
          j->info.status = WF_ESTATE;
          j->err = "cancelled";
          failed += 1;
          continue;
        }
        j->stream = streams.back();
      }
      Status why;
      if (!admit(j, why)) {
        // not enough contiguous arena memory now: release and wait
        for (DevBuf* b : {&j->od.w64, &j->od.w32, &j->od.lam64, &j->od.xlam64, &j->od.xlam32, &j->od.fac64, &j->od.fac32, &j->od.tw64,
                          &j->od.tw32, &j->dw.grid, &j->dw.fine_spec, &j->dw.spec_y, &j->dw.spec_c,
                          &j->dw.tw_fine, &j->xyz_d, &j->nobs, &j->scal, &j->staging, &j->sw.b64,
                          &j->sw.x64, &j->sw.r64, &j->sw.p64, &j->sw.q64, &j->sw.spec64, &j->sw.x32,
                          &j->sw.r32, &j->sw.p32, &j->sw.q32, &j->sw.spec32, &j->sw.bh64, &j->sw.u64, &j->sw.state,
                          &j->sw.partials})
          b->release();
        std::lock_guard<std::mutex> g(mu);
        j->stream = nullptr;
        if (active.empty()) {
          // nothing will free memory: this request cannot run
          queue.pop_front();
          j->phase = FAILED;
          j->info.status = why.code;
          j->err = why.msg;
          failed += 1;
          continue;
        }
        break;
      }
      std::lock_guard<std::mutex> g(mu);
      queue.pop_front();
      streams.pop_back();
      active.push_back(j);
      progressed = true;
    }
    // progress of every admitted request
    std::vector<std::shared_ptr<Job>> act;
    {
      std::lock_guard<std::mutex> g(mu);
      act = active;
    }
    for (auto& j : act) progressed = advance(j) || progressed;
    for (auto& j : act) {
      if (j->phase == DONE || j->phase == FAILED) {
        retire(j, j->phase == DONE);
        std::lock_guard<std::mutex> g(mu);
        active.erase(std::find(active.begin(), active.end(), j));
        progressed = true;
      }
    }
    std::unique_lock<std::mutex> lk(mu);
    if (stop && active.empty() && queue.empty()) break;
    if (!progressed) {
      if (active.empty() && (queue.empty() || stop))
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
    if (hipSetDevice(s->device) != hipSuccess || hipEventCreateWithFlags(&j->ev, hipEventDisableTiming) != hipSuccess)
      return WF_EDEVICE;
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
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) {
    s->err = "unknown ticket";
    return WF_EINVAL;
  }
  const auto& j = it->second;
  const bool fin = (j->phase == DONE || j->phase == FAILED) && j->stream == nullptr;
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
    if (!((j->phase == DONE || j->phase == FAILED) && j->stream == nullptr)) {
      s->err = "request not finished";
      return WF_ESTATE;
    }
    s->jobs.erase(it);
  }
  if (j->phase == FAILED) {
    std::lock_guard<std::mutex> g(s->mu);
    s->err = j->err;
    if (j->ev) (void)hipEventDestroy(j->ev);
    return j->info.status != WF_OK ? (wf_status)j->info.status : WF_EDEVICE;
  }
  std::memcpy(out, j->result.data(), j->result.size() * 8);
  if (j->ev) (void)hipEventDestroy(j->ev);
  return (wf_status)j->info.status;
}

wf_status wf_server_cancel(wf_server* s, uint64_t ticket) {
  if (!s) return WF_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return WF_EINVAL;
  it->second->cancelled = true;
  return WF_OK;
}

wf_status wf_server_stats_get(wf_server* s, wf_server_stats* out) {
  if (!s || !out) return WF_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  *out = wf_server_stats{};
  out->completed = (int64_t)s->latencies.size();
  out->failed = s->failed;
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
  out->peak_bytes = std::max(s->peak.load(), s->arena.peak);
  return WF_OK;
}

const char* wf_server_last_error(const wf_server* s) { return s ? s->err.c_str() : "null server"; }

wf_status wf_server_destroy(wf_server* s) {
  if (!s) return WF_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    for (auto& j : s->queue) j->cancelled = true;
    for (auto& j : s->active) j->cancelled = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto& kv : s->jobs)
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  s->outer.put(s->arena_mem);
  delete s;
  return WF_OK;
}

}  // extern "C"
