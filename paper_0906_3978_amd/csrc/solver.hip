// Conjugate-gradient drivers for the Wiener system A s = b (eq:WF).
//
// FP64: plain CG from s = 0 (Hestenes-Stiefel), stopped on the recursive
// relative residual.
// MIXED: CG with an FP32 operator (FFTs and diagonals) and FP32 vectors, FP64
// dot products, and FP64 "reliable updates" (Sleijpen & van der Vorst): each
// time the recursive FP32 residual has dropped by `delta` since the last
// update, the FP32 correction is folded into the FP64 solution, the residual
// is recomputed as b - A x with the FP64 operator, and the iteration goes on
// from that residual with the same search direction.  This is iterative
// refinement that keeps the Krylov space (a restarted refinement would throw
// it away at every step); convergence is decided on the FP64 residual only.
// Both run several right-hand sides at once when asked: every kernel launch
// covers all of them, each with its own scalars and stop flag.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "checks.h"
#include "solver.h"

namespace wf {

Status validate_opts(const wf_solve_opts& o) {
  wf_status code = WF_OK;
  if (const char* e = opts_error(o, &code)) return fail(code, e);
  return {};
}

double effective_err_tol(const wf_solve_opts& o) {
  if (o.precision != WF_MIXED || o.err_tol < 0.0) return 0.0;
  return o.err_tol > 0.0 ? o.err_tol : DEFAULT_ERR_TOL;
}

int severity(wf_status s) {
  switch (s) {
    case WF_OK: return 0;
    case WF_ENOTCONV: return 1;
    case WF_EBREAKDOWN: return 2;
    default: return 3;
  }
}

namespace {

template <typename T> struct Vecs {
  T *x, *r, *p, *q;
  cplx<T>* spec;
};
Vecs<double> v64(SolveWork& sw) {
  return {sw.x64.as<double>(), sw.r64.as<double>(), sw.p64.as<double>(), sw.q64.as<double>(),
          sw.spec64.as<double2>()};
}
Vecs<float> v32(SolveWork& sw) {
  return {sw.x32.as<float>(), sw.r32.as<float>(), sw.p32.as<float>(), sw.q32.as<float>(),
          sw.spec32.as<float2>()};
}

template <typename T>
Status cg_iteration(const OperatorData& od, SolveWork& sw, Vecs<T> v, int nr, hipStream_t s) {
  CgState* st = sw.state.as<CgState>();
  double* parts = sw.partials.as<double>();
  WF_TRY(operator_passes<T>(od, ZIN_CGP, v.r, v.p, v.x, v.spec, ZOUT_CGQ, v.q, v.p, nullptr, st,
                            parts, nr, SKIP_DONE, s));
  {
    ProfScope ps(od.prof, sizeof(T) == 8 ? WF_PROF_UPDATE_F64 : WF_PROF_UPDATE_F32,
                 3.0 * sizeof(T) * od.g.m * nr, s);
    WF_HIP(launch_cg_update<T>(v.r, v.q, od.g.m, od.g.m, parts, st, nr, s));
  }
  WF_HIP(launch_finalize(FIN_RR, parts, update_blocks(od.g.m, sizeof(T) == 8), SKIP_DONE, st, nr, s));
  return {};
}

// One CG iteration of the prior-split system; vectors are half spectra.
// FP32 (the inner iteration of mixed solves) folds the residual update into
// the first pass of the next iteration: the x pass that forms the direction
// also applies r -= alpha q, and beta comes from p.q and q.q (see
// launch_finalize_fold_pq), which saves the separate update kernel's sweep
// over r and q.  Its q vector keeps only the noise part of C A C p, so that
// the x forward pass need not read p: p.q follows from p.p and, by Parseval,
// from the z middle pass's sum of nbar w u^2.  The iteration in which a
// reliable update falls due has already formed its direction; the update
// continues that direction (see k_rel_reset).
template <typename T>
Status split_iteration(const OperatorData& od, SolveWork& sw, Vecs<T> v, int nr, hipStream_t s) {
  CgState* st = sw.state.as<CgState>();
  double* parts = sw.partials.as<double>();
  if constexpr (sizeof(T) == 4) {
    return split_passes<T>(od, SM_FWD_CGQF, v.p, v.spec, v.q, nullptr, st, parts, nr, SKIP_DONE,
                           s, v.r, v.x);
  } else {
    const int64_t vl = sw.vlen;
    WF_TRY(split_passes<T>(od, SM_FWD_CGQ, v.p, v.spec, v.q, nullptr, st, parts, nr, SKIP_DONE,
                           s, v.r, v.x));
    {
      ProfScope ps(od.prof, WF_PROF_UPDATE_F64, 3.0 * sizeof(T) * vl * nr, s);
      WF_HIP(launch_cg_update<T>(v.r, v.q, vl, vl, parts, st, nr, s));
    }
    WF_HIP(launch_finalize(FIN_RR, parts, update_blocks(vl, true), SKIP_DONE, st, nr, s));
    return {};
  }
}

template <typename T>
Status any_iteration(const OperatorData& od, SolveWork& sw, Vecs<T> v, int nr, hipStream_t s) {
  if (!sw.split) return cg_iteration<T>(od, sw, v, nr, s);
  return split_iteration<T>(od, sw, v, nr, s);
}

// Runs CG iterations in chunks of `check` until every RHS is done.
template <typename T>
Status iterate_until_done(const OperatorData& od, SolveWork& sw, Vecs<T> v, int nr, int check,
                          hipStream_t s) {
  for (;;) {
    WF_TRY(sw.pull_state(s));
    bool all = true;
    for (int i = 0; i < nr; ++i) all = all && sw.st_host[i].done;
    if (all) return {};
    for (int k = 0; k < check; ++k) WF_TRY(any_iteration<T>(od, sw, v, nr, s));
  }
}

// Mixed precision: FP32 iterations until every RHS has stopped; reliable
// updates for the RHS that ask for one.
Status iterate_reliable(const OperatorData& od, SolveWork& sw, int nr, int check, hipStream_t s) {
  Vecs<float> v = v32(sw);
  for (;;) {
    WF_TRY(sw.pull_state(s));
    bool all = true, update = false;
    for (int i = 0; i < nr; ++i) {
      all = all && sw.st_host[i].done;
      update = update || sw.st_host[i].status == CG_UPDATE;
    }
    if (update) {
      WF_TRY(solve_update(od, sw, nr, s));
      continue;
    }
    if (all) return {};
    for (int k = 0; k < check; ++k) WF_TRY(any_iteration<float>(od, sw, v, nr, s));
  }
}

wf_status map_cg_status(int32_t st) {
  switch (st) {
    case CG_CONVERGED: return WF_OK;
    case CG_MAXITER: return WF_ENOTCONV;
    case CG_BREAKDOWN: return WF_EBREAKDOWN;
    case CG_STOPPED: return WF_ENOTCONV;
    default: return WF_ENOTCONV;
  }
}


struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  void start(hipStream_t s) { (void)hipEventRecord(a, s); }
  double stop(hipStream_t s) {
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
};

Status push_states(SolveWork& sw, const std::vector<CgState>& st, hipStream_t s) {
  std::memcpy(sw.st_host, st.data(), sizeof(CgState) * st.size());
  WF_HIP(hipMemcpyAsync(sw.state.p, sw.st_host, sizeof(CgState) * st.size(), hipMemcpyHostToDevice, s));
  WF_HIP(hipStreamSynchronize(s));
  return {};
}

// FP64 CG: applies the pending x += alpha p, then r_true = b - A64 x into
// `out`; outer_rr = ||r_true||^2 per RHS.
Status true_residual(const OperatorData& od, SolveWork& sw, double* out, int nr, hipStream_t s) {
  WF_HIP(launch_cg_flush<double>(sw.x64.as<double>(), sw.p64.as<double>(), od.g.m, od.g.m,
                                 sw.state.as<CgState>(), nr, s));
  return operator_passes<double>(od, ZIN_REAL, sw.x64.as<double>(), nullptr, nullptr,
                                 sw.spec64.as<double2>(), ZOUT_RES, out, sw.x64.as<double>(),
                                 sw.b64.as<double>(), sw.state.as<CgState>(),
                                 sw.partials.as<double>(), nr, SKIP_NONE, s);
}

}  // namespace

Status solve_start(const OperatorData& od, SolveWork& sw, int nr, bool mixed, hipStream_t s) {
  const Grid& g = od.g;
  CgState* st = sw.state.as<CgState>();
  double* parts = sw.partials.as<double>();
  const double* b = sw.b64.as<double>();
  int64_t vl = g.m;
  if (sw.split) {
    if (!od.fac_ready) return fail(WF_ESTATE, "prior-split factor not built");
    // b_hat = C b; onorm = ||b||
    WF_TRY(split_rhs(od, b, sw.spec64.as<double2>(), sw.bh64.as<double>(), nr, s));
    WF_HIP(launch_state_norm(b, g.m, g.m, parts, st, nr, s));
    b = sw.bh64.as<double>();
    vl = sw.vlen;
  }
  if (mixed) {
    WF_HIP(launch_rel_init(sw.x64.as<double>(), sw.r64.as<double>(), b, sw.x32.as<float>(),
                           sw.r32.as<float>(), vl, vl, parts, st, nr, s));
  } else {
    WF_HIP(launch_cg_init<double>(sw.x64.as<double>(), sw.r64.as<double>(), b, vl, vl, parts, st,
                                  nr, s));
  }
  return {};
}

Status solve_chunk(const OperatorData& od, SolveWork& sw, int nr, bool mixed, int iters,
                   hipStream_t s) {
  if (mixed) {
    Vecs<float> v = v32(sw);
    for (int k = 0; k < iters; ++k) WF_TRY(any_iteration<float>(od, sw, v, nr, s));
  } else {
    Vecs<double> v = v64(sw);
    for (int k = 0; k < iters; ++k) WF_TRY(any_iteration<double>(od, sw, v, nr, s));
  }
  return {};
}

Status solve_update(const OperatorData& od, SolveWork& sw, int nr, hipStream_t s) {
  const Grid& g = od.g;
  CgState* st = sw.state.as<CgState>();
  double* parts = sw.partials.as<double>();
  const int64_t vl = sw.split ? sw.vlen : g.m;
  WF_HIP(launch_rel_fold(sw.x64.as<double>(), sw.x32.as<float>(), sw.p32.as<float>(), vl, vl, parts,
                         sw.split ? od.fac64.as<double>() : nullptr, g.n, g.spec_main,
                         od.rhs_fac, st, nr, s));
  if (sw.split) {
    WF_TRY(split_passes<double>(od, SM_FWD_RES, sw.x64.as<double>(), sw.spec64.as<double2>(),
                                sw.r64.as<double>(), sw.bh64.as<double>(), st, parts, nr,
                                SKIP_UNLESS_UPDATE, s));
  } else {
    WF_TRY(operator_passes<double>(od, ZIN_REAL, sw.x64.as<double>(), nullptr, nullptr,
                                   sw.spec64.as<double2>(), ZOUT_RES, sw.r64.as<double>(),
                                   sw.x64.as<double>(), sw.b64.as<double>(), st, parts, nr,
                                   SKIP_UNLESS_UPDATE, s));
  }
  WF_HIP(launch_rel_reset(sw.r32.as<float>(), sw.r64.as<double>(),
                          sw.split ? sw.p32.as<float>() : nullptr, vl, vl, parts, st, nr, s));
  return {};
}

Status solve_finish(const OperatorData& od, SolveWork& sw, int nr, bool mixed, hipStream_t s) {
  if (!sw.split) {
    if (!mixed) WF_TRY(true_residual(od, sw, sw.q64.as<double>(), nr, s));
    return {};
  }
  const int64_t vl = sw.vlen;
  CgState* st = sw.state.as<CgState>();
  if (!mixed)
    WF_HIP(launch_cg_flush<double>(sw.x64.as<double>(), sw.p64.as<double>(), vl, vl, st, nr, s));
  // s = C y into x64 (stride n^3), then ||b - A s||^2 into outer_rr
  WF_TRY(split_solution(od, sw.x64.as<double>(), sw.spec64.as<double2>(), sw.x64.as<double>(), nr,
                        s));
  return operator_passes<double>(od, ZIN_REAL, sw.x64.as<double>(), nullptr, nullptr,
                                 sw.spec64.as<double2>(), ZOUT_RES, sw.u64.as<double>(),
                                 sw.x64.as<double>(), sw.b64.as<double>(), st,
                                 sw.partials.as<double>(), nr, SKIP_NONE, s);
}

void solve_infos(const CgState* st, int nr, bool mixed, bool split, const Grid& g, double ms,
                 wf_solve_info* infos) {
  const double M = (double)g.m;
  for (int i = 0; i < nr; ++i) {
    const CgState& c = st[i];
    wf_solve_info& in = infos[i];
    in = wf_solve_info{};
    in.iters_total = c.iter;
    in.outer_steps = mixed ? c.updates : 0;
    in.rel_res_recursive = c.bnorm > 0 ? c.rel : 0.0;
    const double bn = split ? c.onorm : c.bnorm;
    in.rel_res_true = bn > 0 ? std::sqrt(c.outer_rr) / bn : 0.0;
    in.time_ms = ms;
    // mixed: FP32 iterations; per update: fold (x64 rw, x32 rw), FP64 residual, reset
    const double it = model_bytes_iteration(false, split), it64 = model_bytes_iteration(true, split);
    const double res = model_bytes_residual(split);
    double mb = mixed ? c.iter * it + c.updates * (res + 24.0 + 12.0) + 40.0
                      : c.iter * it64 + (split ? 0.0 : model_bytes_residual(false));
    // split: C b and ||b|| at the start; C y and ||b - A s|| at the end
    if (split) mb += 3 * 16.0 + 8.0 + 3 * 16.0 + model_bytes_residual(false);
    in.model_bytes = mb * M;
    in.nbar = c.nbar;
    in.status = map_cg_status(c.status);
    in.last_change = mixed ? c.move : 0.0;
    in.stagnated = c.stagnated;
  }
}

Status run_solve(const SolveRequest& rq, wf_solve_info* infos) {
  const OperatorData& od = *rq.od;
  const Grid& g = od.g;
  SolveWork& sw = *rq.work;
  const int nr = rq.nrhs;
  const hipStream_t s = rq.stream;
  const wf_solve_opts& o = rq.opts;
  const bool mixed = o.precision == WF_MIXED;
  const bool split = o.precond == WF_PRECOND_PRIOR;
  const int check = o.check_every > 0 ? o.check_every : 16;
  WF_TRY(sw.ensure(*rq.al, g, nr, !mixed, mixed, split));
  std::vector<CgState> st(nr);
  for (int i = 0; i < nr; ++i) {
    st[i] = CgState{};
    st[i].nbar = rq.nbar[i];
    st[i].tol = o.tol;
    st[i].max_iter = o.max_iter;
    st[i].delta = o.inner_tol > 0 ? o.inner_tol : 0.1;
    st[i].max_updates = o.max_outer;
    st[i].err_tol = effective_err_tol(o);
    st[i].hold_need = settle_intervals(st[i].delta);
  }
  WF_TRY(push_states(sw, st, s));
  Timer tm;
  tm.start(s);
  WF_TRY(solve_start(od, sw, nr, mixed, s));
  if (mixed) WF_TRY(iterate_reliable(od, sw, nr, check, s));
  else WF_TRY(iterate_until_done<double>(od, sw, v64(sw), nr, check, s));
  WF_TRY(solve_finish(od, sw, nr, mixed, s));
  const double ms = tm.stop(s);
  WF_TRY(sw.pull_state(s));
  solve_infos(sw.st_host, nr, mixed, split, g, ms, infos);
  Status worst{};
  for (int i = 0; i < nr; ++i) {
    const wf_status stt = (wf_status)infos[i].status;
    if (severity(stt) > severity(worst.code))
      worst = fail(stt, std::string("rhs ") + std::to_string(i) + ": " + wf_status_str(stt));
  }
  return worst;
}

// ---- stepwise solve (checkpoint / resume) ---------------------------------

Status step_begin(const OperatorData& od, const Allocator& al, SolveWork& sw, double nbar,
                  const wf_solve_opts& o, hipStream_t s) {
  const bool mixed = o.precision == WF_MIXED;
  WF_TRY(sw.ensure(al, od.g, 1, !mixed, mixed, o.precond == WF_PRECOND_PRIOR));
  std::vector<CgState> st(1);
  st[0] = CgState{};
  st[0].nbar = nbar;
  st[0].tol = o.tol;
  st[0].max_iter = o.max_iter;
  st[0].delta = o.inner_tol > 0 ? o.inner_tol : 0.1;
  st[0].max_updates = o.max_outer;
  st[0].err_tol = effective_err_tol(o);
  st[0].hold_need = settle_intervals(st[0].delta);
  WF_TRY(push_states(sw, st, s));
  return solve_start(od, sw, 1, mixed, s);
}

Status step_iterations(const OperatorData& od, SolveWork& sw, int iters, bool mixed,
                       hipStream_t s) {
  if (!mixed) {
    Vecs<double> v = v64(sw);
    for (int k = 0; k < iters; ++k) WF_TRY(any_iteration<double>(od, sw, v, 1, s));
    return {};
  }
  // FP32 iterations until `iters` more have run or the solve stops, with the
  // reliable updates the state asks for on the way (the device decides when;
  // how the host chunks its launches changes nothing).  The folded
  // prior-split iteration ends with its step pending, counted by the next
  // one: a pending step counts as done here.
  WF_TRY(sw.pull_state(s));
  const bool fold = sw.split;
  auto steps = [fold](const CgState& c) {
    return (int64_t)c.iter + (fold && c.pending && !c.done ? 1 : 0);
  };
  const int64_t target = steps(sw.st_host[0]) + iters;
  Vecs<float> v = v32(sw);
  for (;;) {
    const CgState& c = sw.st_host[0];
    if (steps(c) >= target) return {};
    if (c.status == CG_UPDATE) {
      WF_TRY(solve_update(od, sw, 1, s));
    } else if (c.done) {
      return {};
    } else {
      const int64_t left = target - steps(c);
      for (int64_t k = 0; k < std::min<int64_t>(left, 16); ++k)
        WF_TRY(any_iteration<float>(od, sw, v, 1, s));
    }
    WF_TRY(sw.pull_state(s));
  }
}

Status step_finish(const OperatorData& od, SolveWork& sw, bool mixed, hipStream_t s,
                   wf_solve_info* info) {
  WF_TRY(sw.pull_state(s));
  if (mixed && !sw.st_host[0].done) {
    // stopped between reliable updates: fold the FP32 correction and take the
    // FP64 residual, as an update would (the solve may find itself converged)
    WF_HIP(launch_state_request_update(sw.state.as<CgState>(), s));
    WF_TRY(solve_update(od, sw, 1, s));
    WF_TRY(sw.pull_state(s));
  }
  const bool stopped = sw.st_host[0].done != 0;
  WF_TRY(solve_finish(od, sw, 1, mixed, s));
  WF_TRY(sw.pull_state(s));
  const CgState& c = sw.st_host[0];
  solve_infos(sw.st_host, 1, mixed, sw.split, od.g, 0.0, info);
  info->status = stopped ? map_cg_status(c.status) : WF_ENOTCONV;
  if (info->status != WF_OK)
    return fail((wf_status)info->status, wf_status_str((wf_status)info->status));
  return {};
}

namespace {
struct SnapHeader {
  uint64_t magic;
  int32_t n;
  int32_t split;  // 1: prior-split solve (the vectors are half spectra)
  double box;
  int32_t mixed;  // 1: mixed precision (FP64 x, r; FP32 x, r, p and, prior-split, q)
  int32_t pad;
};
constexpr uint64_t SNAP_MAGIC = 0x5746534e41503034ull;  // "WFSNAP04"
}  // namespace

static size_t vector_len(const Grid& g, bool split) {
  return split ? 2 * (size_t)g.spec_total : (size_t)g.m;
}

size_t snapshot_bytes(const Grid& g, bool split, bool mixed) {
  const size_t v = vector_len(g, split);
  return sizeof(SnapHeader) + sizeof(CgState) +
         (mixed ? 2 * v * 8 + (split ? 4 : 3) * v * 4 : 3 * v * 8);
}

bool snapshot_kind(const void* buf, bool* split, bool* mixed) {
  SnapHeader h;
  std::memcpy(&h, buf, sizeof h);
  if (h.magic != SNAP_MAGIC) return false;
  *split = h.split == 1;
  *mixed = h.mixed == 1;
  return true;
}

// the device vectors of a snapshot, in order, and their element sizes (the
// folded FP32 prior-split iteration keeps r -= alpha q pending between
// iterations, so its snapshot holds q as well)
static std::vector<std::pair<DevBuf*, size_t>> snap_vectors(SolveWork& sw, bool mixed) {
  if (mixed && sw.split)
    return {{&sw.x64, 8}, {&sw.r64, 8}, {&sw.x32, 4}, {&sw.r32, 4}, {&sw.p32, 4}, {&sw.q32, 4}};
  if (mixed) return {{&sw.x64, 8}, {&sw.r64, 8}, {&sw.x32, 4}, {&sw.r32, 4}, {&sw.p32, 4}};
  return {{&sw.x64, 8}, {&sw.r64, 8}, {&sw.p64, 8}};
}

Status snapshot_save(const Grid& g, SolveWork& sw, bool mixed, void* buf, hipStream_t s) {
  char* p = static_cast<char*>(buf);
  SnapHeader h{SNAP_MAGIC, g.n, sw.split ? 1 : 0, g.box, mixed ? 1 : 0, 0};
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  WF_HIP(hipMemcpyAsync(p, sw.state.p, sizeof(CgState), hipMemcpyDeviceToHost, s));
  p += sizeof(CgState);
  const size_t v = vector_len(g, sw.split);
  for (auto& [b, es] : snap_vectors(sw, mixed)) {
    WF_HIP(hipMemcpyAsync(p, b->p, v * es, hipMemcpyDeviceToHost, s));
    p += v * es;
  }
  WF_HIP(hipStreamSynchronize(s));
  return {};
}

Status snapshot_load(const OperatorData& od, const Allocator& al, SolveWork& sw, const void* buf,
                     hipStream_t s) {
  const char* p = static_cast<const char*>(buf);
  SnapHeader h;
  std::memcpy(&h, p, sizeof h);
  if (h.magic != SNAP_MAGIC || h.n != od.g.n || h.box != od.g.box || (h.split != 0 && h.split != 1) ||
      (h.mixed != 0 && h.mixed != 1))
    return fail(WF_EINVAL, "snapshot does not match this grid");
  const bool split = h.split == 1, mixed = h.mixed == 1;
  if (split && !od.fac_ready) return fail(WF_ESTATE, "prior-split factor not built");
  WF_TRY(sw.ensure(al, od.g, 1, !mixed, mixed, split));
  p += sizeof h;
  CgState st;
  std::memcpy(&st, p, sizeof st);
  st.ticket = 0;
  WF_HIP(hipMemcpyAsync(sw.state.p, &st, sizeof st, hipMemcpyHostToDevice, s));
  p += sizeof(CgState);
  const size_t v = vector_len(od.g, split);
  for (auto& [b, es] : snap_vectors(sw, mixed)) {
    WF_HIP(hipMemcpyAsync(b->p, p, v * es, hipMemcpyHostToDevice, s));
    p += v * es;
  }
  // the prior-split right-hand side C b of the reliable updates, recomputed
  // from the context's data vector (the same bits as at the start)
  if (split && mixed)
    WF_TRY(split_rhs(od, sw.b64.as<double>(), sw.spec64.as<double2>(), sw.bh64.as<double>(), 1,
                     s));
  WF_HIP(hipStreamSynchronize(s));
  return {};
}

// ---- multi-RHS batch ---------------------------------------------------------

Status run_batch(const OperatorData& od, const Allocator& al, DepositWork& dw,
                 const BatchInputs& bi, const wf_solve_opts& o, double* const* s_out,
                 wf_solve_info* infos, double sumw, hipStream_t s) {
  const Grid& g = od.g;
  const int nr = bi.nrhs;
  SolveWork sw;
  WF_TRY(sw.ensure(al, g, nr, o.precision == WF_FP64, o.precision == WF_MIXED,
                   o.precond == WF_PRECOND_PRIOR));
  DevBuf xyz, nobs, scal, flag;
  WF_TRY(nobs.ensure(al, (size_t)g.m * 8));
  WF_TRY(scal.ensure(al, (size_t)(2 + nr) * 8));
  WF_TRY(flag.ensure(al, 256));
  WF_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  WF_HIP(hipMemcpyAsync(scal.p, &sumw, 8, hipMemcpyHostToDevice, s));
  for (int i = 0; i < nr; ++i) {
    const double* src = bi.xyz[i];
    const int64_t ng = bi.n_gal[i];
    if (bi.mem == WF_HOST) {
      WF_TRY(xyz.ensure(al, (size_t)std::max<int64_t>(ng, 1) * 24));
      WF_TRY(upload(xyz.p, bi.xyz[i], (size_t)ng * 24, WF_HOST, s));
      src = xyz.as<double>();
    }
    WF_HIP(launch_check_xyz(src, ng, g.box, flag.as<int>(), s));
    WF_TRY(run_deposit(al, od, dw, src, ng, bi.scheme, bi.ss, nobs.as<double>(), s));
    WF_HIP(launch_data_vector(nobs.as<double>(), od.w64.as<double>(), scal.as<double>(), (double)ng,
                              scal.as<double>() + 2 + i, sw.b64.as<double>() + (size_t)i * g.m, g.m,
                              s));
  }
  dw.fine_spec.release();
  dw.spec_y.release();
  dw.spec_c.release();
  int bad = 0;
  std::vector<double> nbar(nr);
  WF_HIP(hipMemcpyAsync(&bad, flag.p, sizeof bad, hipMemcpyDeviceToHost, s));
  WF_HIP(hipMemcpyAsync(nbar.data(), scal.as<double>() + 2, 8 * (size_t)nr, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  if (bad) return fail(WF_EINVAL, "galaxy coordinates must satisfy 0 <= x < L");
  SolveRequest rq;
  rq.od = &od;
  rq.al = &al;
  rq.work = &sw;
  rq.nrhs = nr;
  rq.nbar = nbar.data();
  rq.opts = o;
  rq.stream = s;
  Status r = run_solve(rq, infos);
  if (r.code == WF_OK || r.code == WF_ENOTCONV || r.code == WF_EBREAKDOWN) {
    for (int i = 0; i < nr; ++i)
      WF_TRY(download(s_out[i], sw.x64.as<double>() + (size_t)i * g.m, (size_t)g.m * 8, bi.mem, s));
    WF_HIP(hipStreamSynchronize(s));
  }
  return r;
}

size_t footprint_bytes(int n, int ss, wf_precision prec, int nrhs, bool split) {
  if (n <= 0 || nrhs <= 0 || (ss != 1 && ss != 2)) return 0;
  Grid g;
  g.set(n, 1.0);
  const double M = (double)g.m, ST = (double)g.spec_total;
  const double V = split ? 2.0 * ST : M;  // elements of one CG vector
  double op = 12.0 * M + 8.0 * g.lamlen + 12.0 * g.xlamlen + 24.0 * n;
  if (split) op += 12.0 * (double)split_fac_elems(n);
  double per = 8.0 * M + 16.0 * V + 16.0 * ST;              // b, x, r, spec64
  per += prec == WF_FP64 ? 16.0 * V : 16.0 * V + 8.0 * ST;  // p, q | 4 FP32 vectors, spec32
  if (split) per += 8.0 * V + 8.0 * M;  // C b, a real field
  const int nf = ss * n;
  double dep = 8.0 * (double)nf * nf * nf + 8.0 * M;  // integer grid, n_obs
  if (ss == 2)
    dep += 16.0 * ((double)nf * nf * (n / 2) + (double)nf * n * (n / 2) + ST) + 16.0 * nf;
  const double parts = 8.0 * std::max<double>((double)g.nrows / 2, 2048.0) * nrhs;
  return (size_t)(op + per * nrhs + dep + parts + 4096.0 * nrhs);
}

}  // namespace wf
