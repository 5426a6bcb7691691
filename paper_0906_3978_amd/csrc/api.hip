// The C ABI of include/wiener.h: context, inputs, gridding, operator test
// hooks and the FP64 / mixed-precision conjugate-gradient solves.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "internal.h"
#include "solver.h"

using namespace wf;

struct wf_ctx {
  Allocator al;
  hipStream_t stream = nullptr;
  std::string err;
  OperatorData od;
  bool have_grid = false, have_mask = false, have_power = false, have_gal = false;
  bool have_rhs = false;
  bool dep_current = false;  // n^o and nbar belong to the current galaxies and mask
  DevBuf xyz, nobs, scal, flag, mpartials;
  int64_t n_gal = 0;
  double sumw = 0.0, nbar = 0.0;
  int dep_scheme = -1, dep_ss = 0;
  DepositWork dw;
  SolveWork sw;
  bool solve_active = false;
  bool active_mixed = false;
  wf_solve_opts active_opts{};
  double active_ms = 0.0;
  Profiler prof;
};

namespace {

wf_status finish(wf_ctx* c, const Status& s) {
  if (!s.ok()) c->err = s.msg;
  return s.code;
}

Status set_device(const wf_ctx* c) {
  WF_HIP(hipSetDevice(c->al.device));
  return {};
}

bool n_supported(int n) {
  if (n < 8 || n > 512) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  if (m != 1 && m != 3) return false;
  return fft_length_supported(n, false) && fft_length_supported(2 * n, true);
}

Status read_flag(wf_ctx* c, int* out) {
  WF_HIP(hipMemcpyAsync(out, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  WF_HIP(hipStreamSynchronize(c->stream));
  return {};
}

Status clear_flag(wf_ctx* c) {
  WF_HIP(hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  return {};
}

Status need(bool cond, const char* what) {
  if (!cond) return fail(WF_ESTATE, what);
  return {};
}

}  // namespace

extern "C" {

int wf_abi_version(void) { return WF_ABI_VERSION; }

const char* wf_status_str(wf_status s) {
  switch (s) {
    case WF_OK: return "ok";
    case WF_EINVAL: return "invalid argument";
    case WF_ESTATE: return "call out of order";
    case WF_ENOMEM: return "out of device memory";
    case WF_EDEVICE: return "HIP runtime error";
    case WF_ENOTCONV: return "not converged within max_iter";
    case WF_EOVERFLOW: return "too many galaxies for exact accumulation";
    case WF_EBREAKDOWN: return "CG breakdown (operator not SPD)";
  }
  return "unknown status";
}

const char* wf_last_error(const wf_ctx* c) { return c ? c->err.c_str() : "null context"; }

wf_status wf_ctx_create(wf_ctx** out, int device, void* hip_stream, wf_alloc_fn alloc,
                        wf_free_fn free_fn, void* user) {
  if (!out) return WF_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return WF_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return WF_EDEVICE;
  }
  wf_ctx* c = new (std::nothrow) wf_ctx();
  if (!c) return WF_ENOMEM;
  c->al.alloc = alloc;
  c->al.free_fn = free_fn;
  c->al.user = user;
  c->al.device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  Status s = set_device(c);
  if (s.ok()) s = c->flag.ensure(c->al, 256);
  if (s.ok()) s = c->scal.ensure(c->al, 64 * sizeof(double));
  if (!s.ok()) {
    delete c;
    return s.code;
  }
  *out = c;
  return WF_OK;
}

wf_status wf_ctx_destroy(wf_ctx* c) {
  if (!c) return WF_EINVAL;
  (void)hipSetDevice(c->al.device);
  (void)hipStreamSynchronize(c->stream);
  delete c;
  return WF_OK;
}

wf_status wf_set_grid(wf_ctx* c, int32_t n, double box) {
  if (!c) return WF_EINVAL;
  if (!n_supported(n)) return finish(c, fail(WF_EINVAL, "n must be 2^a 3^b (b <= 1), 8 <= n <= 512"));
  if (!(box > 0.0) || !std::isfinite(box)) return finish(c, fail(WF_EINVAL, "box must be finite and > 0"));
  Status s = set_device(c);
  if (s.ok()) {
    c->od.g.set(n, box);
    c->have_grid = c->have_mask = c->have_power = c->have_gal = c->have_rhs = false;
    c->dep_current = false;
    c->od.fac_ready = false;
    c->solve_active = false;
    c->dep_scheme = -1;
    s = make_twiddles(c->al, n, c->od.tw64, &c->od.tw32, c->stream);
  }
  if (s.ok()) c->have_grid = true;
  return finish(c, s);
}

wf_status wf_set_mask(wf_ctx* c, const double* w, wf_mem mem) {
  if (!c || !w) return c ? finish(c, fail(WF_EINVAL, "null mask")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  const Grid& g = c->od.g;
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    DevBuf staging;
    const double* src = w;
    if (mem == WF_HOST) {
      WF_TRY(staging.ensure(c->al, (size_t)g.m * 8));
      WF_TRY(upload(staging.p, w, (size_t)g.m * 8, WF_HOST, c->stream));
      src = staging.as<double>();
    }
    WF_TRY(c->od.w64.ensure(c->al, (size_t)g.m * 8));
    WF_TRY(c->od.w32.ensure(c->al, (size_t)g.m * 4));
    WF_TRY(c->mpartials.ensure(c->al, 4096 * 8));
    WF_TRY(clear_flag(c));
    WF_HIP(hipMemsetAsync(c->scal.p, 0, 64 * sizeof(double), c->stream));
    // ticket lives in scal[8]
    WF_HIP(launch_mask(src, c->od.w64.as<double>(), c->od.w32.as<float>(), g.m, c->flag.as<int>(),
                       c->mpartials.as<double>(), reinterpret_cast<uint32_t*>(c->scal.as<double>() + 8),
                       c->scal.as<double>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    double sumw = 0.0;
    WF_HIP(hipMemcpy(&sumw, c->scal.p, 8, hipMemcpyDeviceToHost));
    if (bad) return fail(WF_EINVAL, "mask values must be finite and in [0, 1]");
    if (!(sumw > 0.0)) return fail(WF_EINVAL, "mask is zero everywhere");
    c->sumw = sumw;
    return {};
  };
  s = run();
  c->have_mask = s.ok();
  c->dep_current = false;
  c->have_rhs = false;
  return finish(c, s);
}

wf_status wf_set_power(wf_ctx* c, const double* p, int64_t len, wf_mem mem) {
  if (!c || !p) return c ? finish(c, fail(WF_EINVAL, "null spectrum")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  const Grid& g = c->od.g;
  if (len != g.lamlen)
    return finish(c, fail(WF_EINVAL, "p_by_m2 length must be 3 (n/2)^2 + 1 = " + std::to_string(g.lamlen)));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    DevBuf staging;
    const double* src = p;
    if (mem == WF_HOST) {
      WF_TRY(staging.ensure(c->al, (size_t)len * 8));
      WF_TRY(upload(staging.p, p, (size_t)len * 8, WF_HOST, c->stream));
      src = staging.as<double>();
    }
    c->od.fac_ready = false;
    WF_TRY(c->od.lam64.ensure(c->al, (size_t)len * 8));
    WF_TRY(alloc_xlam(c->al, c->od));
    WF_TRY(clear_flag(c));
    const double h = g.box / g.n;
    WF_HIP(launch_lambda(src, len, h * h * h, 1.0 / (double)g.m, c->od.lam64.as<double>(),
                         c->flag.as<int>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    if (bad) return fail(WF_EINVAL, "P(k) must be finite and > 0 for j >= 1");
    return build_xlam(c->od, c->stream);
  };
  s = run();
  c->have_power = s.ok();
  return finish(c, s);
}

wf_status wf_set_galaxies(wf_ctx* c, const double* xyz, int64_t n_gal, wf_mem mem) {
  if (!c) return WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  if (n_gal < 0 || (n_gal > 0 && !xyz)) return finish(c, fail(WF_EINVAL, "bad galaxy array"));
  if (n_gal >= (int64_t(1) << 24))
    return finish(c, fail(WF_EOVERFLOW, "n_gal must be < 2^24 for exact int64 accumulation"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    WF_TRY(c->xyz.ensure(c->al, (size_t)std::max<int64_t>(n_gal, 1) * 24));
    WF_TRY(upload(c->xyz.p, xyz, (size_t)n_gal * 24, mem, c->stream));
    WF_TRY(clear_flag(c));
    WF_HIP(launch_check_xyz(c->xyz.as<double>(), n_gal, c->od.g.box, c->flag.as<int>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    if (bad) return fail(WF_EINVAL, "galaxy coordinates must satisfy 0 <= x < L");
    c->n_gal = n_gal;
    return {};
  };
  s = run();
  c->have_gal = s.ok();
  c->dep_current = false;
  return finish(c, s);
}

wf_status wf_deposit(wf_ctx* c, wf_scheme scheme, int32_t ss) {
  if (!c) return WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_gal,
                  "wf_deposit needs wf_set_grid, wf_set_mask and wf_set_galaxies");
  if (!s.ok()) return finish(c, s);
  if (scheme < WF_NGP || scheme > WF_TSC) return finish(c, fail(WF_EINVAL, "unknown scheme"));
  if (ss != 1 && ss != 2) return finish(c, fail(WF_EINVAL, "supersample must be 1 or 2"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    WF_TRY(c->nobs.ensure(c->al, (size_t)g.m * 8));
    WF_TRY(c->sw.b64.ensure(c->al, (size_t)g.m * 8));
    WF_TRY(run_deposit(c->al, c->od, c->dw, c->xyz.as<double>(), c->n_gal, scheme, ss,
                       c->nobs.as<double>(), c->stream));
    // drop the transient spectra of the supersampling step
    c->dw.fine_spec.release();
    c->dw.spec_y.release();
    c->dw.spec_c.release();
    // sumw sits in scal[0]; nbar goes to scal[1]
    WF_HIP(hipMemcpyAsync(c->scal.p, &c->sumw, 8, hipMemcpyHostToDevice, c->stream));
    WF_HIP(launch_data_vector(c->nobs.as<double>(), c->od.w64.as<double>(), c->scal.as<double>(),
                              (double)c->n_gal, c->scal.as<double>() + 1, c->sw.b64.as<double>(),
                              g.m, c->stream));
    double nbar = 0.0;
    WF_HIP(hipMemcpyAsync(&nbar, c->scal.as<double>() + 1, 8, hipMemcpyDeviceToHost, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    c->nbar = nbar;
    c->dep_scheme = scheme;
    c->dep_ss = ss;
    return {};
  };
  s = run();
  c->have_rhs = s.ok();
  c->dep_current = s.ok();
  c->solve_active = false;
  return finish(c, s);
}

wf_status wf_get_deposit(wf_ctx* c, int64_t* fine, double* nobs, double* nbar, wf_mem mem) {
  if (!c) return WF_EINVAL;
  Status s = need(c->dep_scheme >= 0, "no deposit yet");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    const int nf = c->dep_ss * g.n;
    if (fine) WF_TRY(download(fine, c->dw.grid.p, (size_t)nf * nf * nf * 8, mem, c->stream));
    if (nobs) WF_TRY(download(nobs, c->nobs.p, (size_t)g.m * 8, mem, c->stream));
    if (nbar) {
      if (mem == WF_HOST) *nbar = c->nbar;
      else WF_TRY(download(nbar, c->scal.as<double>() + 1, 8, mem, c->stream));
    }
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_set_rhs(wf_ctx* c, const double* b, double nbar, wf_mem mem) {
  if (!c || !b) return c ? finish(c, fail(WF_EINVAL, "null rhs")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  if (!(nbar > 0.0) || !std::isfinite(nbar)) return finish(c, fail(WF_EINVAL, "nbar must be > 0"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    WF_TRY(c->sw.b64.ensure(c->al, (size_t)g.m * 8));
    WF_TRY(upload(c->sw.b64.p, b, (size_t)g.m * 8, mem, c->stream));
    c->nbar = nbar;
    return {};
  };
  s = run();
  c->have_rhs = s.ok();
  c->dep_current = false;
  c->solve_active = false;
  return finish(c, s);
}

wf_status wf_apply_operator(wf_ctx* c, wf_precision prec, const double* v, double* av,
                            wf_mem mem) {
  if (!c || !v || !av) return c ? finish(c, fail(WF_EINVAL, "null vector")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_power && c->have_rhs,
                  "operator needs grid, mask, power and nbar");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    SolveWork& sw = c->sw;
    WF_TRY(sw.ensure(c->al, g, 1, true, prec == WF_MIXED));
    CgState st{};
    st.nbar = c->nbar;
    WF_HIP(hipMemcpyAsync(sw.state.p, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    WF_TRY(upload(sw.x64.p, v, (size_t)g.m * 8, mem, c->stream));
    if (prec == WF_FP64) {
      WF_TRY(operator_passes<double>(c->od, ZIN_REAL, sw.x64.as<double>(), nullptr, nullptr,
                                     sw.spec64.as<double2>(), ZOUT_APPLY, sw.q64.as<double>(),
                                     sw.x64.as<double>(), nullptr, sw.state.as<CgState>(),
                                     sw.partials.as<double>(), 1, SKIP_NONE, c->stream));
    } else {
      WF_HIP(launch_f64_to_f32(sw.x32.as<float>(), sw.x64.as<double>(), g.m, c->stream));
      WF_TRY(operator_passes<float>(c->od, ZIN_REAL, sw.x32.as<float>(), nullptr, nullptr,
                                    sw.spec32.as<float2>(), ZOUT_APPLY, sw.q32.as<float>(),
                                    sw.x32.as<float>(), nullptr, sw.state.as<CgState>(),
                                    sw.partials.as<double>(), 1, SKIP_NONE, c->stream));
      WF_HIP(launch_f32_to_f64(sw.q64.as<double>(), sw.q32.as<float>(), g.m, c->stream));
    }
    WF_TRY(download(av, sw.q64.p, (size_t)g.m * 8, mem, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_forward_spectrum(wf_ctx* c, wf_precision prec, const double* v, double* spec,
                              wf_mem mem) {
  if (!c || !v || !spec) return c ? finish(c, fail(WF_EINVAL, "null vector")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    SolveWork& sw = c->sw;
    WF_TRY(sw.ensure(c->al, g, 1, true, prec == WF_MIXED));
    WF_TRY(upload(sw.x64.p, v, (size_t)g.m * 8, mem, c->stream));
    const int h = g.n / 2;
    std::vector<double> main_h, nyq_h;
    if (prec == WF_FP64) {
      WF_TRY(forward_passes<double>(c->od, sw.x64.as<double>(), sw.spec64.as<double2>(), c->stream));
      main_h.resize((size_t)g.spec_total * 2);
      WF_HIP(hipMemcpyAsync(main_h.data(), sw.spec64.p, main_h.size() * 8, hipMemcpyDeviceToHost,
                            c->stream));
      WF_HIP(hipStreamSynchronize(c->stream));
    } else {
      WF_HIP(launch_f64_to_f32(sw.x32.as<float>(), sw.x64.as<double>(), g.m, c->stream));
      WF_TRY(forward_passes<float>(c->od, sw.x32.as<float>(), sw.spec32.as<float2>(), c->stream));
      std::vector<float> tmp((size_t)g.spec_total * 2);
      WF_HIP(hipMemcpyAsync(tmp.data(), sw.spec32.p, tmp.size() * 4, hipMemcpyDeviceToHost, c->stream));
      WF_HIP(hipStreamSynchronize(c->stream));
      main_h.assign(tmp.begin(), tmp.end());
    }
    // assemble numpy's rfftn layout [n][n][n/2+1]
    std::vector<double> out((size_t)g.nrows * (h + 1) * 2);
    const double* nyq = main_h.data() + (size_t)g.spec_main * 2;
    for (int64_t row = 0; row < g.nrows; ++row) {
      std::memcpy(&out[(size_t)row * (h + 1) * 2], &main_h[(size_t)row * h * 2], (size_t)h * 16);
      out[((size_t)row * (h + 1) + h) * 2] = nyq[row * 2];
      out[((size_t)row * (h + 1) + h) * 2 + 1] = nyq[row * 2 + 1];
    }
    WF_TRY(download(spec, nullptr, 0, mem, c->stream));
    if (mem == WF_HOST) std::memcpy(spec, out.data(), out.size() * 8);
    else WF_HIP(hipMemcpy(spec, out.data(), out.size() * 8, hipMemcpyHostToDevice));
    return {};
  };
  return finish(c, run());
}

// ---- solves ----------------------------------------------------------------

wf_status wf_solve(wf_ctx* c, const wf_solve_opts* opts, double* s_out, wf_mem mem,
                   wf_solve_info* info) {
  if (!c || !opts || !s_out) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_power && c->have_rhs,
                  "wf_solve needs grid, mask, power and a data vector");
  if (!s.ok()) return finish(c, s);
  s = validate_opts(*opts);
  if (!s.ok()) return finish(c, s);
  s = set_device(c);
  if (s.ok() && opts->precond == WF_PRECOND_PRIOR) s = ensure_split_fac(c->al, c->od, c->stream);
  if (!s.ok()) return finish(c, s);
  SolveRequest rq;
  rq.od = &c->od;
  rq.al = &c->al;
  rq.work = &c->sw;
  rq.nrhs = 1;
  rq.nbar = &c->nbar;
  rq.opts = *opts;
  rq.stream = c->stream;
  std::vector<wf_solve_info> infos(1);
  Status r = run_solve(rq, infos.data());
  if (r.code == WF_OK || r.code == WF_ENOTCONV) {
    Status d = download(s_out, c->sw.x64.p, (size_t)c->od.g.m * 8, mem, c->stream);
    if (!d.ok()) return finish(c, d);
    Status sy = [&]() -> Status { WF_HIP(hipStreamSynchronize(c->stream)); return {}; }();
    if (!sy.ok()) return finish(c, sy);
  }
  if (info) *info = infos[0];
  return finish(c, r);
}

// ---- checkpoint / resume of an FP64 solve ------------------------------------

wf_status wf_solve_begin(wf_ctx* c, const wf_solve_opts* opts) {
  if (!c || !opts) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_power && c->have_rhs,
                  "wf_solve_begin needs grid, mask, power and a data vector");
  if (!s.ok()) return finish(c, s);
  s = validate_opts(*opts);
  if (s.ok()) s = set_device(c);
  if (s.ok() && opts->precond == WF_PRECOND_PRIOR) s = ensure_split_fac(c->al, c->od, c->stream);
  if (s.ok()) s = step_begin(c->od, c->al, c->sw, c->nbar, *opts, c->stream);
  c->solve_active = s.ok();
  c->active_mixed = opts->precision == WF_MIXED;
  c->active_opts = *opts;
  c->active_ms = 0.0;
  return finish(c, s);
}

wf_status wf_solve_step(wf_ctx* c, int32_t iters, int32_t* done) {
  if (!c || iters < 0) return c ? finish(c, fail(WF_EINVAL, "bad iteration count")) : WF_EINVAL;
  Status s = need(c->solve_active, "wf_solve_begin or wf_solve_resume first");
  if (!s.ok()) return finish(c, s);
  s = set_device(c);
  if (s.ok()) s = step_iterations(c->od, c->sw, iters, c->active_mixed, c->stream);
  if (s.ok()) s = c->sw.pull_state(c->stream);
  if (s.ok() && done) *done = c->sw.st_host[0].done;
  return finish(c, s);
}

size_t wf_snapshot_bytes(const wf_ctx* c) {
  if (!c || !c->have_grid) return 0;
  return snapshot_bytes(c->od.g, c->solve_active && c->sw.split,
                        c->solve_active && c->active_mixed);
}

wf_status wf_solve_snapshot(wf_ctx* c, void* buf, size_t bytes) {
  if (!c || !buf) return c ? finish(c, fail(WF_EINVAL, "null buffer")) : WF_EINVAL;
  Status s = need(c->solve_active, "no active solve");
  if (!s.ok()) return finish(c, s);
  if (bytes < snapshot_bytes(c->od.g, c->sw.split, c->active_mixed))
    return finish(c, fail(WF_EINVAL, "snapshot buffer too small"));
  s = set_device(c);
  if (s.ok()) s = snapshot_save(c->od.g, c->sw, c->active_mixed, buf, c->stream);
  return finish(c, s);
}

wf_status wf_solve_resume(wf_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf) return c ? finish(c, fail(WF_EINVAL, "null buffer")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_power && c->have_rhs,
                  "resume needs grid, mask, power and a data vector");
  if (!s.ok()) return finish(c, s);
  bool split = false, mixed = false;
  if (bytes < snapshot_bytes(c->od.g, false, false) || !snapshot_kind(buf, &split, &mixed))
    return finish(c, fail(WF_EINVAL, "not a snapshot of this library"));
  if (bytes < snapshot_bytes(c->od.g, split, mixed))
    return finish(c, fail(WF_EINVAL, "snapshot buffer too small"));
  s = set_device(c);
  if (s.ok() && split) s = ensure_split_fac(c->al, c->od, c->stream);
  if (s.ok()) s = snapshot_load(c->od, c->al, c->sw, buf, c->stream);
  c->solve_active = s.ok();
  c->active_mixed = mixed;
  return finish(c, s);
}

wf_status wf_solve_finish(wf_ctx* c, double* s_out, wf_mem mem, wf_solve_info* info) {
  if (!c || !s_out) return c ? finish(c, fail(WF_EINVAL, "null output")) : WF_EINVAL;
  Status s = need(c->solve_active, "no active solve");
  if (!s.ok()) return finish(c, s);
  wf_solve_info inf{};
  s = set_device(c);
  if (s.ok()) s = step_finish(c->od, c->sw, c->active_mixed, c->stream, &inf);
  if (s.ok() || s.code == WF_ENOTCONV) {
    Status d = download(s_out, c->sw.x64.p, (size_t)c->od.g.m * 8, mem, c->stream);
    if (!d.ok()) return finish(c, d);
  }
  if (info) *info = inf;
  c->solve_active = false;
  return finish(c, s);
}

wf_status wf_solve_batch(wf_ctx* c, int32_t nrhs, const double* const* xyz, const int64_t* n_gal,
                         wf_scheme scheme, int32_t ss, const wf_solve_opts* opts,
                         double* const* s_out, wf_mem mem, wf_solve_info* infos) {
  if (!c) return WF_EINVAL;
  if (nrhs <= 0 || !xyz || !n_gal || !opts || !s_out)
    return finish(c, fail(WF_EINVAL, "bad batch arguments"));
  Status s = need(c->have_grid && c->have_mask && c->have_power, "batch needs grid, mask and power");
  if (!s.ok()) return finish(c, s);
  s = validate_opts(*opts);
  if (!s.ok()) return finish(c, s);
  if (scheme < WF_NGP || scheme > WF_TSC || (ss != 1 && ss != 2))
    return finish(c, fail(WF_EINVAL, "bad scheme or supersample"));
  for (int i = 0; i < nrhs; ++i) {
    if (n_gal[i] < 0 || (n_gal[i] > 0 && !xyz[i]) || !s_out[i])
      return finish(c, fail(WF_EINVAL, "bad catalogue " + std::to_string(i)));
    if (n_gal[i] >= (int64_t(1) << 24))
      return finish(c, fail(WF_EOVERFLOW, "n_gal must be < 2^24"));
  }
  s = set_device(c);
  if (s.ok() && opts->precond == WF_PRECOND_PRIOR) s = ensure_split_fac(c->al, c->od, c->stream);
  if (!s.ok()) return finish(c, s);
  BatchInputs bi;
  bi.nrhs = nrhs;
  bi.xyz = xyz;
  bi.n_gal = n_gal;
  bi.scheme = scheme;
  bi.ss = ss;
  bi.mem = mem;
  std::vector<wf_solve_info> inf(nrhs);
  s = run_batch(c->od, c->al, c->dw, bi, *opts, s_out, inf.data(), c->sumw, c->stream);
  if (infos)
    for (int i = 0; i < nrhs; ++i) infos[i] = inf[i];
  c->have_rhs = false;
  c->solve_active = false;
  return finish(c, s);
}

// ---- signal-dependent noise ----------------------------------------------------

wf_status wf_jackknife_counts(wf_ctx* c, double alpha, uint64_t seed, int64_t first,
                              int32_t count, int32_t* out, wf_mem mem) {
  if (!c || !out) return c ? finish(c, fail(WF_EINVAL, "null output")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_gal,
                  "needs wf_set_grid, wf_set_mask and wf_set_galaxies");
  if (!s.ok()) return finish(c, s);
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return finish(c, fail(WF_EINVAL, "alpha must be > 0"));
  if (count <= 0 || first < 0) return finish(c, fail(WF_EINVAL, "need count > 0 and first >= 0"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    DevBuf tmp;
    int32_t* dst = reinterpret_cast<int32_t*>(out);
    if (mem == WF_HOST) {
      WF_TRY(tmp.ensure(c->al, (size_t)count * g.m * 4));
      dst = tmp.as<int32_t>();
    }
    WF_HIP(hipMemsetAsync(dst, 0, (size_t)count * g.m * 4, c->stream));
    WF_TRY(clear_flag(c));
    WF_HIP(launch_sd_counts(true, c->xyz.as<double>(), c->n_gal, (double)g.n / g.box, g.n,
                            c->od.w64.as<double>(), alpha, seed, first, count, dst,
                            c->flag.as<int>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    if (bad) return fail(WF_EINVAL, "alpha exceeds w at the node of a galaxy");
    if (mem == WF_HOST) WF_TRY(download(out, dst, (size_t)count * g.m * 4, WF_HOST, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_solve_sd(wf_ctx* c, const wf_solve_opts* opts, int32_t kind, double alpha,
                      uint64_t seed, int64_t first, int32_t nsamples, double* mean_out,
                      double* samples_out, wf_mem mem, wf_solve_info* infos) {
  if (!c || !opts || !mean_out) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_power && c->have_gal && c->dep_current,
                  "wf_solve_sd needs grid, mask, power, galaxies and a wf_deposit of them");
  if (!s.ok()) return finish(c, s);
  s = validate_opts(*opts);
  if (!s.ok()) return finish(c, s);
  if (kind == WF_NOISE_SD_MEAN) {
    if (nsamples != 1) return finish(c, fail(WF_EINVAL, "the mean estimator has one sample"));
  } else if (kind == WF_NOISE_SD_JACKKNIFE) {
    if (nsamples <= 0 || first < 0) return finish(c, fail(WF_EINVAL, "need nsamples > 0, first >= 0"));
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return finish(c, fail(WF_EINVAL, "alpha must be > 0"));
  } else {
    return finish(c, fail(WF_EINVAL, "unknown noise kind"));
  }
  s = set_device(c);
  if (s.ok() && opts->precond == WF_PRECOND_PRIOR) s = ensure_split_fac(c->al, c->od, c->stream);
  if (!s.ok()) return finish(c, s);
  SdRequest rq;
  rq.od = &c->od;
  rq.al = &c->al;
  rq.xyz = c->xyz.as<double>();
  rq.n_gal = c->n_gal;
  rq.nobs = c->nobs.as<double>();
  rq.nbar = c->nbar;
  rq.kind = kind;
  rq.alpha = alpha;
  rq.seed = seed;
  rq.first = first;
  rq.nsamples = nsamples;
  rq.opts = *opts;
  rq.mean_out = mean_out;
  rq.samples_out = samples_out;
  rq.mem = mem;
  rq.flag = c->flag.as<int>();
  rq.stream = c->stream;
  std::vector<wf_solve_info> inf(nsamples);
  s = run_sd(rq, inf.data());
  if (infos)
    for (int i = 0; i < nsamples; ++i) infos[i] = inf[i];
  c->solve_active = false;
  return finish(c, s);
}

// ---- after the solve ---------------------------------------------------------

wf_status wf_rsd_factor(wf_ctx* c, double beta, double sigma, double* out, int64_t len,
                        wf_mem mem) {
  if (!c || !out) return c ? finish(c, fail(WF_EINVAL, "null output")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  const Grid& g = c->od.g;
  if (len <= 0 || len > g.lamlen) return finish(c, fail(WF_EINVAL, "len must be in [1, 3 (n/2)^2 + 1]"));
  if (!std::isfinite(beta) || !(sigma >= 0.0) || !std::isfinite(sigma))
    return finish(c, fail(WF_EINVAL, "beta must be finite and sigma >= 0"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    DevBuf tmp;
    double* dst = out;
    if (mem == WF_HOST) {
      WF_TRY(tmp.ensure(c->al, (size_t)len * 8));
      dst = tmp.as<double>();
    }
    const double dk = 2.0 * M_PI / g.box;
    WF_HIP(launch_rsd_factor(dk * dk, beta, sigma, dst, len, c->stream));
    if (mem == WF_HOST) WF_TRY(download(out, dst, (size_t)len * 8, WF_HOST, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_fourier_filter(wf_ctx* c, int32_t kind, double a, double b, double cc,
                            const double* table, int64_t len, const double* in, double* out,
                            wf_mem mem) {
  if (!c || !in || !out) return c ? finish(c, fail(WF_EINVAL, "null field")) : WF_EINVAL;
  Status s = need(c->have_grid, "wf_set_grid first");
  if (!s.ok()) return finish(c, s);
  const Grid& g = c->od.g;
  if (kind == WF_FILTER_TABLE) {
    if (!table || len != g.lamlen)
      return finish(c, fail(WF_EINVAL, "table length must be 3 (n/2)^2 + 1 = " + std::to_string(g.lamlen)));
  } else if (kind == WF_FILTER_GAUSS) {
    if (!(a >= 0.0) || !std::isfinite(a)) return finish(c, fail(WF_EINVAL, "r_S must be >= 0"));
  } else if (kind == WF_FILTER_RSD_DECONV) {
    if (!std::isfinite(a) || !(b >= 0.0) || !std::isfinite(b) || !(cc > 0.0) || !std::isfinite(cc))
      return finish(c, fail(WF_EINVAL, "need finite beta, sigma >= 0 and bias > 0"));
  } else {
    return finish(c, fail(WF_EINVAL, "unknown filter kind"));
  }
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    DevBuf h, rows64, rows32, field, spec, tab;
    WF_TRY(h.ensure(c->al, (size_t)g.lamlen * 8));
    const double* tdev = nullptr;
    if (kind == WF_FILTER_TABLE) {
      if (mem == WF_HOST) {
        WF_TRY(tab.ensure(c->al, (size_t)g.lamlen * 8));
        WF_TRY(upload(tab.p, table, (size_t)g.lamlen * 8, WF_HOST, c->stream));
        tdev = tab.as<double>();
      } else {
        tdev = table;
      }
    }
    WF_TRY(clear_flag(c));
    const double dk = 2.0 * M_PI / g.box;
    WF_HIP(launch_filter_table(kind, dk * dk, a, b, cc, tdev, g.lamlen, 1.0 / (double)g.m,
                               h.as<double>(), c->flag.as<int>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    if (bad) return fail(WF_EINVAL, "the filter is not finite everywhere");
    WF_TRY(rows64.ensure(c->al, (size_t)g.xlamlen * 8));
    WF_TRY(rows32.ensure(c->al, (size_t)g.xlamlen * 4));
    WF_HIP(launch_xlam_rows(g.n, h.as<double>(), rows64.as<double>(), rows32.as<float>(), c->stream));
    rows32.release();
    WF_TRY(spec.ensure(c->al, (size_t)g.spec_total * 16));
    const double* src = in;
    double* dst = out;
    if (mem == WF_HOST) {
      WF_TRY(field.ensure(c->al, (size_t)g.m * 8));
      WF_TRY(upload(field.p, in, (size_t)g.m * 8, WF_HOST, c->stream));
      src = dst = field.as<double>();
    }
    WF_TRY(filter_passes(c->od, rows64.as<double>(), src, spec.as<double2>(), dst, c->stream));
    if (mem == WF_HOST) WF_TRY(download(out, dst, (size_t)g.m * 8, WF_HOST, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_field_moments(wf_ctx* c, const double* v, int32_t masked, double* out5, wf_mem mem) {
  if (!c || !v || !out5) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && (!masked || c->have_mask), "needs the grid (and mask)");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    DevBuf field;
    const double* src = v;
    if (mem == WF_HOST) {
      WF_TRY(field.ensure(c->al, (size_t)g.m * 8));
      WF_TRY(upload(field.p, v, (size_t)g.m * 8, WF_HOST, c->stream));
      src = field.as<double>();
    }
    double sm[5];
    WF_TRY(field_sums(src, masked ? c->od.w64.as<double>() : nullptr, g.m, c->mpartials, c->al, sm,
                      c->stream));
    moments_from_sums(sm, out5);
    return {};
  };
  return finish(c, run());
}

wf_status wf_field_moments_noalloc(wf_ctx* c, const double* v, int32_t masked, double* out5) {
  if (!c || !v || !out5) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && (!masked || c->have_mask), "needs the grid (and mask)");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    // a host pointer reaching the kernel would fault the GPU: refuse it here
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, v) != hipSuccess) {
      (void)hipGetLastError();
      return fail(WF_EINVAL, "v must be device memory on the context's GPU");
    }
    if ((at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) ||
        at.device != c->al.device)
      return fail(WF_EINVAL, "v must be device memory on the context's GPU");
    double sm[5];
    WF_TRY(field_sums_noalloc(v, masked ? c->od.w64.as<double>() : nullptr, c->od.g.m,
                              c->al.device, sm, c->stream));
    moments_from_sums(sm, out5);
    return {};
  };
  return finish(c, run());
}

wf_status wf_compare_fields(wf_ctx* c, const double* rec, const double* tru, int32_t masked,
                            double* out3, wf_mem mem) {
  if (!c || !rec || !tru || !out3) return c ? finish(c, fail(WF_EINVAL, "null argument")) : WF_EINVAL;
  Status s = need(c->have_grid && (!masked || c->have_mask), "needs the grid (and mask)");
  if (!s.ok()) return finish(c, s);
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    DevBuf fr, ft, flag;
    const double *r = rec, *t = tru;
    if (mem == WF_HOST) {
      WF_TRY(fr.ensure(c->al, (size_t)g.m * 8));
      WF_TRY(ft.ensure(c->al, (size_t)g.m * 8));
      WF_TRY(upload(fr.p, rec, (size_t)g.m * 8, WF_HOST, c->stream));
      WF_TRY(upload(ft.p, tru, (size_t)g.m * 8, WF_HOST, c->stream));
      r = fr.as<double>();
      t = ft.as<double>();
    }
    double sm[6];
    bool kl_ok = true;
    WF_TRY(compare_sums(r, t, masked ? c->od.w64.as<double>() : nullptr, g.m, c->mpartials, flag,
                        c->al, sm, &kl_ok, c->stream));
    const double n = sm[5];
    out3[0] = (sm[1] > 0 && sm[2] > 0) ? sm[0] / (std::sqrt(sm[1]) * std::sqrt(sm[2])) : NAN;
    out3[1] = n > 0 ? std::sqrt(sm[3] / n) : NAN;
    out3[2] = (n > 0 && kl_ok) ? sm[4] / n : NAN;
    return {};
  };
  return finish(c, run());
}

wf_status wf_inverse_weighting(wf_ctx* c, wf_scheme scheme, int32_t ss, double* out, wf_mem mem) {
  if (!c || !out) return c ? finish(c, fail(WF_EINVAL, "null output")) : WF_EINVAL;
  Status s = need(c->have_grid && c->have_mask && c->have_gal,
                  "needs wf_set_grid, wf_set_mask and wf_set_galaxies");
  if (!s.ok()) return finish(c, s);
  if (scheme < WF_NGP || scheme > WF_TSC) return finish(c, fail(WF_EINVAL, "unknown scheme"));
  if (ss != 1 && ss != 2) return finish(c, fail(WF_EINVAL, "supersample must be 1 or 2"));
  auto run = [&]() -> Status {
    WF_TRY(set_device(c));
    const Grid& g = c->od.g;
    const int nf = ss * g.n;
    const int64_t mf = (int64_t)nf * nf * nf;
    DevBuf fine, field;
    WF_TRY(fine.ensure(c->al, (size_t)mf * 8));
    WF_HIP(launch_fill_f64(fine.as<double>(), mf, c->stream));
    WF_TRY(clear_flag(c));
    WF_HIP(launch_deposit_iw(scheme, c->xyz.as<double>(), c->n_gal, (double)nf / g.box, nf,
                             (double)g.n / g.box, g.n, c->od.w64.as<double>(), fine.as<double>(),
                             c->flag.as<int>(), c->stream));
    int bad = 0;
    WF_TRY(read_flag(c, &bad));
    if (bad) return fail(WF_EINVAL, "a galaxy lies on a node with w = 0");
    double* dst = out;
    if (mem == WF_HOST) {
      WF_TRY(field.ensure(c->al, (size_t)g.m * 8));
      dst = field.as<double>();
    }
    WF_TRY(run_lowpass(c->al, c->od, c->dw, nullptr, fine.as<double>(), 1.0, ss, dst, c->stream));
    c->dw.fine_spec.release();
    c->dw.spec_y.release();
    c->dw.spec_c.release();
    fine.release();
    // nbar of eq:nmean
    const double nbar = c->sumw > 0 ? (double)c->n_gal / c->sumw : 0.0;
    if (!(nbar > 0.0)) return fail(WF_EINVAL, "no galaxies: nbar = 0");
    WF_HIP(launch_overdensity(dst, g.m, 1.0 / nbar, c->stream));
    if (mem == WF_HOST) WF_TRY(download(out, dst, (size_t)g.m * 8, WF_HOST, c->stream));
    WF_HIP(hipStreamSynchronize(c->stream));
    return {};
  };
  return finish(c, run());
}

wf_status wf_profile_enable(wf_ctx* c, int32_t on) {
  if (!c) return WF_EINVAL;
  if (on < 0) return finish(c, fail(WF_EINVAL, "profile_enable: negative sampling period"));
  Status s = set_device(c);
  if (!s.ok()) return finish(c, s);
  (void)hipStreamSynchronize(c->stream);
  c->prof.harvest();
  c->prof.clear();
  c->prof.on = on != 0;
  c->prof.every = on > 1 ? on : 1;
  c->od.prof = c->prof.on ? &c->prof : nullptr;
  return WF_OK;
}

wf_status wf_profile_read(wf_ctx* c, wf_profile* out) {
  if (!c || !out) return c ? finish(c, fail(WF_EINVAL, "null output")) : WF_EINVAL;
  Status s = set_device(c);
  if (!s.ok()) return finish(c, s);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return finish(c, fail(WF_EDEVICE, "sync failed"));
  c->prof.harvest();
  c->prof.totals(out->launches, out->skipped, out->ms, out->bytes);
  return WF_OK;
}

size_t wf_footprint_bytes(int32_t n, int32_t ss, wf_precision prec, int32_t nrhs) {
  return std::max(footprint_bytes(n, ss, prec, nrhs, false), footprint_bytes(n, ss, prec, nrhs, true));
}

}  // extern "C"
