// Host-side building blocks: device memory, twiddles, the operator pipeline
// and the gridding pipeline.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace wf {

void* Allocator::get(size_t bytes) const {
  if (bytes == 0) bytes = 256;
  if (alloc) return alloc(bytes, user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Allocator::put(void* p) const {
  if (!p) return;
  if (free_fn) free_fn(p, user);
  else (void)hipFree(p);
}

void DevBuf::release() {
  if (p && a) a->put(p);
  p = nullptr;
  bytes = 0;
}

Status DevBuf::ensure(const Allocator& al, size_t b) {
  if (p && bytes >= b && a == &al) return {};
  release();
  a = &al;
  p = al.get(b);
  if (!p) return fail(WF_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
  bytes = b;
  return {};
}

Profiler::~Profiler() {
  for (auto& pr : pending) {
    (void)hipEventDestroy(pr.a);
    (void)hipEventDestroy(pr.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

void Profiler::clear() {
  for (int k = 0; k < WF_PROF_KINDS; ++k) {
    dur[k].clear();
    byt[k].clear();
    seen[k] = 0;
  }
}

void Profiler::totals(int64_t* launches, int64_t* skipped, double* ms, double* bytes) const {
  for (int k = 0; k < WF_PROF_KINDS; ++k) {
    launches[k] = skipped[k] = 0;
    ms[k] = bytes[k] = 0.0;
    if (dur[k].empty()) continue;
    std::vector<float> t = dur[k];
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    const float cut = 0.8f * t[t.size() / 2];
    for (size_t i = 0; i < dur[k].size(); ++i) {
      if (dur[k][i] < cut) {
        skipped[k] += 1;
        continue;
      }
      launches[k] += 1;
      ms[k] += dur[k][i];
      bytes[k] += byt[k][i];
    }
  }
}

TimedLaunch& timed_launch() {
  static thread_local TimedLaunch t;
  return t;
}

int Profiler::begin(int kind, double b, hipStream_t s, bool multi) {
  if (!on) return -1;
  if (seen[kind]++ % every != 0) return -1;
  if (pending.size() >= 8192) {
    (void)hipStreamSynchronize(s);
    harvest();
  }
  hipEvent_t e[2];
  for (auto& x : e) {
    if (!pool.empty()) {
      x = pool.back();
      pool.pop_back();
    } else if (hipEventCreateWithFlags(&x, hipEventDisableSystemFence) != hipSuccess) {
      return -1;
    }
  }
  if (multi) {
    (void)hipEventRecord(e[0], s);
  } else {
    TimedLaunch& t = timed_launch();
    t.start = e[0];
    t.stop = e[1];
  }
  pending.push_back(Pair{e[0], e[1], kind, b});
  return (int)pending.size() - 1;
}

void Profiler::end(int idx, hipStream_t s, bool multi) {
  if (multi) {
    (void)hipEventRecord(pending[idx].b, s);
    return;
  }
  TimedLaunch& t = timed_launch();
  if (t.start == pending[idx].a) {  // nothing was launched (an early error return)
    t.start = t.stop = nullptr;
    pool.push_back(pending[idx].a);
    pool.push_back(pending[idx].b);
    pending.erase(pending.begin() + idx);
  }
}

void Profiler::harvest() {
  for (auto& pr : pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pr.a, pr.b) == hipSuccess) {
      dur[pr.kind].push_back(t);
      byt[pr.kind].push_back(pr.bytes);
    }
    pool.push_back(pr.a);
    pool.push_back(pr.b);
  }
  pending.clear();
}

void Grid::set(int n_, double box_) {
  n = n_;
  box = box_;
  m = (int64_t)n * n * n;
  nrows = (int64_t)n * n;
  spec_main = (int64_t)n * n * (n / 2);
  spec_total = spec_main + (int64_t)n * n;
  lamlen = 3 * (int64_t)(n / 2) * (n / 2) + 1;
  xlamlen = xlam_elems(n);
}

Status alloc_xlam(const Allocator& al, OperatorData& od) {
  WF_TRY(od.xlam64.ensure(al, (size_t)od.g.xlamlen * 8));
  WF_TRY(od.xlam32.ensure(al, (size_t)od.g.xlamlen * 4));
  return {};
}

Status build_xlam(OperatorData& od, hipStream_t s) {
  WF_HIP(launch_xlam_rows(od.g.n, od.lam64.as<double>(), od.xlam64.as<double>(),
                          od.xlam32.as<float>(), s));
  return {};
}

SolveWork::~SolveWork() {
  if (st_host && !view) (void)hipHostFree(st_host);
}

static void alias_part(DevBuf& dst, const DevBuf& src, size_t per, int slot) {
  if (src.p) dst.alias(static_cast<char*>(src.p) + per * slot, per);
  else dst.release();
}

void SolveWork::make_view(const SolveWork& src, const Grid& g, int slot) {
  view = true;
  nrhs = 1;
  split = src.split;
  vlen = src.vlen;
  const size_t m = (size_t)g.m, v = (size_t)vlen, sp = (size_t)g.spec_total;
  alias_part(b64, src.b64, m * 8, slot);
  alias_part(x64, src.x64, v * 8, slot);
  alias_part(r64, src.r64, v * 8, slot);
  alias_part(p64, src.p64, v * 8, slot);
  alias_part(q64, src.q64, v * 8, slot);
  alias_part(spec64, src.spec64, sp * 16, slot);
  alias_part(x32, src.x32, v * 4, slot);
  alias_part(r32, src.r32, v * 4, slot);
  alias_part(p32, src.p32, v * 4, slot);
  alias_part(q32, src.q32, v * 4, slot);
  alias_part(spec32, src.spec32, sp * 8, slot);
  alias_part(bh64, src.bh64, v * 8, slot);
  alias_part(u64, src.u64, m * 8, slot);
  alias_part(state, src.state, sizeof(CgState), slot);
  partials.alias(src.partials.p, src.partials.bytes);
  st_host = src.st_host + slot;
  st_cap = 1;
}

void OperatorData::make_view(const OperatorData& src, int slot, double box) {
  g = src.g;
  g.box = box;
  alias_part(w64, src.w64, (size_t)src.rhs_w * 8, slot);
  alias_part(w32, src.w32, (size_t)src.rhs_w * 4, slot);
  tw64.alias(src.tw64.p, src.tw64.bytes);
  tw32.alias(src.tw32.p, src.tw32.bytes);
  alias_part(lam64, src.lam64, (size_t)src.rhs_lam * 8, slot);
  alias_part(xlam64, src.xlam64, (size_t)src.rhs_xlam * 8, slot);
  alias_part(xlam32, src.xlam32, (size_t)src.rhs_xlam * 4, slot);
  alias_part(fac64, src.fac64, (size_t)src.rhs_fac * 8, slot);
  alias_part(fac32, src.fac32, (size_t)src.rhs_fac * 4, slot);
  fac_ready = src.fac_ready;
  sd = false;
  prof = src.prof;
  rhs_w = rhs_lam = rhs_xlam = rhs_fac = 0;
}

Status SolveWork::ensure(const Allocator& al, const Grid& g, int nr, bool fp64_cg, bool mixed,
                         bool split_) {
  nrhs = nr;
  split = split_;
  vlen = split ? 2 * g.spec_total : g.m;
  const size_t m = (size_t)g.m * nr;
  const size_t v = (size_t)vlen * nr;
  const size_t sp = (size_t)g.spec_total * nr;
  WF_TRY(b64.ensure(al, m * 8));
  WF_TRY(x64.ensure(al, v * 8));
  WF_TRY(r64.ensure(al, v * 8));
  WF_TRY(spec64.ensure(al, sp * 16));
  if (fp64_cg) {
    WF_TRY(p64.ensure(al, v * 8));
    WF_TRY(q64.ensure(al, v * 8));
  }
  if (mixed) {
    WF_TRY(x32.ensure(al, v * 4));
    WF_TRY(r32.ensure(al, v * 4));
    WF_TRY(p32.ensure(al, v * 4));
    WF_TRY(q32.ensure(al, v * 4));
    WF_TRY(spec32.ensure(al, sp * 8));
  }
  if (split) {
    WF_TRY(bh64.ensure(al, v * 8));
    WF_TRY(u64.ensure(al, m * 8));
  }
  // partials: enough for the largest grid of any reduction kernel per RHS
  const int64_t per = partials_per_rhs(g);
  WF_TRY(partials.ensure(al, (size_t)per * nr * 8));
  WF_TRY(state.ensure(al, sizeof(CgState) * nr));
  if (st_cap < nr) {
    if (st_host) (void)hipHostFree(st_host);
    st_host = nullptr;
    WF_HIP(hipHostMalloc((void**)&st_host, sizeof(CgState) * nr, hipHostMallocDefault));
    st_cap = nr;
  }
  return {};
}

int64_t partials_per_rhs(const Grid& g) {
  const int64_t zblocks = g.nrows / 2;  // upper bound of z-pass blocks (NB >= 1)
  return std::max<int64_t>(zblocks, 4096);
}

Status SolveWork::pull_state(hipStream_t s) {
  WF_HIP(hipMemcpyAsync(st_host, state.p, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  return {};
}

Status make_twiddles(const Allocator& al, int n, DevBuf& tw64, DevBuf* tw32, hipStream_t st) {
  std::vector<double> t(2 * (size_t)n);
  std::vector<float> f(2 * (size_t)n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < n; ++m) {
    // exp(-2 pi i m / n), reduced to the first octant for accuracy
    long double ang = (long double)two_pi * (long double)m / (long double)n;
    double c = (double)cosl(ang), s = -(double)sinl(ang);
    if (4 * m == n) { c = 0.0; s = -1.0; }
    if (2 * m == n) { c = -1.0; s = 0.0; }
    if (4 * m == 3 * n) { c = 0.0; s = 1.0; }
    if (m == 0) { c = 1.0; s = 0.0; }
    t[2 * m] = c;
    t[2 * m + 1] = s;
    f[2 * m] = (float)c;
    f[2 * m + 1] = (float)s;
  }
  WF_TRY(tw64.ensure(al, t.size() * 8));
  WF_HIP(hipMemcpyAsync(tw64.p, t.data(), t.size() * 8, hipMemcpyHostToDevice, st));
  if (tw32) {
    WF_TRY(tw32->ensure(al, f.size() * 4));
    WF_HIP(hipMemcpyAsync(tw32->p, f.data(), f.size() * 4, hipMemcpyHostToDevice, st));
  }
  WF_HIP(hipStreamSynchronize(st));  // the host tables go out of scope
  return {};
}

Status upload(void* dst, const void* src, size_t bytes, wf_mem mem, hipStream_t s) {
  if (bytes == 0) return {};
  WF_HIP(hipMemcpyAsync(dst, src, bytes,
                        mem == WF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
  if (mem == WF_HOST) WF_HIP(hipStreamSynchronize(s));
  return {};
}

Status download(void* dst, const void* src, size_t bytes, wf_mem mem, hipStream_t s) {
  if (bytes == 0) return {};
  WF_HIP(hipMemcpyAsync(dst, src, bytes,
                        mem == WF_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  if (mem == WF_HOST) WF_HIP(hipStreamSynchronize(s));
  return {};
}

// ---------------------------------------------------------------------------
// segment descriptors of the strided passes
// ---------------------------------------------------------------------------
template <typename T> static Seg<T> seg_y_main(cplx<T>* spec, const Grid& g, int tb) {
  Seg<T> s{};
  const int64_t h = g.n / 2;
  s.in = spec;
  s.out = spec;
  s.in_outer = s.out_outer = g.n * h;
  s.in_axis = s.out_axis = h;
  s.in_batch = s.out_batch = 1;
  s.in_rhs = s.out_rhs = g.spec_total;
  s.n_outer = g.n;
  s.n_btiles = (int)(h / tb);
  s.n_out = g.n;
  return s;
}
template <typename T> static Seg<T> seg_y_nyq(cplx<T>* nyq, const Grid& g, int tb) {
  Seg<T> s{};
  s.in = nyq;
  s.out = nyq;
  s.in_axis = s.out_axis = 1;
  s.in_batch = s.out_batch = g.n;
  s.in_rhs = s.out_rhs = g.spec_total;
  s.n_outer = 1;
  s.n_btiles = g.n / tb;
  s.axis_contig = 1;
  s.n_out = g.n;
  return s;
}
template <typename T> static Seg<T> seg_x_main(cplx<T>* spec, const Grid& g, int tb) {
  Seg<T> s{};
  const int64_t h = g.n / 2;
  s.in = spec;
  s.out = spec;
  s.in_outer = s.out_outer = h;
  s.in_axis = s.out_axis = g.n * h;
  s.in_batch = s.out_batch = 1;
  s.in_rhs = s.out_rhs = g.spec_total;
  s.n_outer = g.n;
  s.n_btiles = (int)(h / tb);
  s.n_out = g.n;
  s.lam_y_outer = 1;
  s.lam_kz = -1;
  return s;
}
template <typename T> static Seg<T> seg_x_nyq(cplx<T>* nyq, const Grid& g, int tb) {
  Seg<T> s{};
  s.in = nyq;
  s.out = nyq;
  s.in_axis = s.out_axis = g.n;
  s.in_batch = s.out_batch = 1;
  s.in_rhs = s.out_rhs = g.spec_total;
  s.n_outer = 1;
  s.n_btiles = g.n / tb;
  s.n_out = g.n;
  s.lam_y_outer = 0;
  s.lam_kz = g.n / 2;
  return s;
}

template <typename T> static const cplx<T>* tw_of(const OperatorData& od) {
  if constexpr (sizeof(T) == 8) return od.tw64.as<cplx<T>>();
  else return od.tw32.as<cplx<T>>();
}
template <typename T> static const T* lam_of(const OperatorData& od) {
  if constexpr (sizeof(T) == 8) return od.xlam64.as<T>();
  else return od.xlam32.as<T>();
}
template <typename T> static const T* w_of(const OperatorData& od) {
  if constexpr (sizeof(T) == 8) return od.w64.as<T>();
  else return od.w32.as<T>();
}
// the noise diagonal of the operator: nbar w (the mask, shared by all RHS, times
// each RHS's nbar) or the per-RHS signal-dependent arrays nbar w g
template <typename T, typename Args> static void set_noise_diag(const OperatorData& od, Args& a) {
  if (od.sd) {
    if constexpr (sizeof(T) == 8) a.w = od.dg64.as<T>();
    else a.w = od.dg32.as<T>();
    a.rhs_w = od.g.m;
    a.w_scaled = 1;
  } else {
    a.w = w_of<T>(od);
    a.rhs_w = od.rhs_w;
    a.w_scaled = 0;
  }
}

template <typename T>
static StrArgs<T> str_args(const OperatorData& od, cplx<T>* spec, bool xpass, const CgState* st,
                           int skip) {
  const Grid& g = od.g;
  const int tb = strided_tb(g.n, sizeof(T) == 8);
  cplx<T>* nyq = spec + g.spec_main;
  StrArgs<T> a{};
  a.s0 = xpass ? seg_x_main<T>(spec, g, tb) : seg_y_main<T>(spec, g, tb);
  a.s1 = xpass ? seg_x_nyq<T>(nyq, g, tb) : seg_y_nyq<T>(nyq, g, tb);
  a.nblk0 = a.s0.n_outer * a.s0.n_btiles;
  a.nblk1 = a.s1.n_outer * a.s1.n_btiles;
  a.lam = lam_of<T>(od);
  a.rhs_lam = od.rhs_xlam;
  a.tw = tw_of<T>(od);
  a.st = skip != SKIP_NONE ? st : nullptr;
  a.skip = skip;
  return a;
}

template <typename T>
StrArgs<T> spectrum_args(const OperatorData& od, cplx<T>* spec, bool xpass) {
  return str_args<T>(od, spec, xpass, nullptr, SKIP_NONE);
}
template StrArgs<float> spectrum_args<float>(const OperatorData&, cplx<float>*, bool);
template StrArgs<double> spectrum_args<double>(const OperatorData&, cplx<double>*, bool);

template <typename T>
Status operator_passes(const OperatorData& od, int zin_mode, const T* in_or_r, T* p, T* x,
                       cplx<T>* spec, int zout_mode, T* out, const T* aux, const double* bvec,
                       CgState* st, double* partials, int nrhs, int skip, hipStream_t s) {
  const Grid& g = od.g;
  const int kbase = sizeof(T) == 8 ? WF_PROF_ZFWD_F64 : WF_PROF_ZFWD_F32;
  const double vb = (double)sizeof(T) * g.m * nrhs;                 // one real vector
  const double sb = 2.0 * sizeof(T) * g.spec_total * nrhs;         // one half spectrum
  ZfwdArgs<T> zf{};
  zf.in = in_or_r;
  zf.p = p;
  zf.x = x;
  zf.out_main = spec;
  zf.out_nyq = spec + g.spec_main;
  zf.nkz_out = g.n / 2;
  zf.rhs_in = g.m;
  zf.rhs_main = g.spec_total;
  zf.rhs_nyq = g.spec_total;
  zf.tw = tw_of<T>(od);
  zf.st = (zin_mode == ZIN_CGP || skip != SKIP_NONE) ? st : nullptr;
  zf.skip = skip;
  {
    // CG: r, p, x in; p, x, spectrum out
    ProfScope ps(od.prof, kbase + 0, (zin_mode == ZIN_CGP ? 5 * vb : vb) + sb, s);
    WF_HIP(launch_zfwd<T>(g.n, zin_mode, zf, g.nrows, nrhs, s));
  }
  {
    ProfScope ps(od.prof, kbase + 1, 2 * sb, s);
    WF_HIP(launch_strided<T>(g.n, SM_FWD, str_args<T>(od, spec, false, st, skip), nrhs, s));
  }
  {
    // spectrum in and out, one Lambda value per element
    ProfScope ps(od.prof, kbase + 2, 2.5 * sb, s);
    WF_HIP(launch_strided<T>(g.n, SM_FWD_LAM_INV, str_args<T>(od, spec, true, st, skip), nrhs, s));
  }
  {
    ProfScope ps(od.prof, kbase + 3, 2 * sb, s);
    WF_HIP(launch_strided<T>(g.n, SM_INV, str_args<T>(od, spec, false, st, skip), nrhs, s));
  }
  ZinvArgs<T> zi{};
  zi.in_main = spec;
  zi.in_nyq = spec + g.spec_main;
  zi.rhs_main = g.spec_total;
  zi.rhs_nyq = g.spec_total;
  zi.out = out;
  zi.rhs_out = g.m;
  zi.aux = aux;
  zi.rhs_aux = g.m;
  set_noise_diag<T>(od, zi);
  zi.bvec = bvec;
  zi.rhs_b = g.m;
  zi.scale = 1.0;
  zi.partials = partials;
  zi.tw = tw_of<T>(od);
  zi.st = st;
  zi.skip = skip;
  {
    // spectrum in; aux and the noise diagonal in (the mask once for all RHS, SD
    // arrays per RHS); result out; RES also reads b
    const double wb = (double)sizeof(T) * g.m * (od.sd ? nrhs : 1);
    double zb = sb + 2 * vb + wb;
    if (zout_mode == ZOUT_RES) zb += 8.0 * g.m * nrhs;
    {
      ProfScope ps(od.prof, kbase + 4, zb, s);
      WF_HIP(launch_zinv<T>(g.n, zout_mode, zi, g.nrows, nrhs, s));
    }
    if (zout_mode == ZOUT_CGQ || zout_mode == ZOUT_RES)
      WF_HIP(launch_finalize(zout_mode == ZOUT_CGQ ? FIN_PQ : FIN_RES, partials,
                             zpass_blocks(g.n, g.nrows, sizeof(T) == 8), skip, st, nrhs, s));
  }
  return {};
}

template Status operator_passes<float>(const OperatorData&, int, const float*, float*, float*,
                                       cplx<float>*, int, float*, const float*, const double*,
                                       CgState*, double*, int, int, hipStream_t);
template Status operator_passes<double>(const OperatorData&, int, const double*, double*, double*,
                                        cplx<double>*, int, double*, const double*, const double*,
                                        CgState*, double*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// prior-split operator (C A C) on half-spectrum vectors
// ---------------------------------------------------------------------------
Status alloc_split_fac(const Allocator& al, OperatorData& od) {
  const int64_t len = split_fac_elems(od.g.n);
  WF_TRY(od.fac64.ensure(al, (size_t)len * 8));
  WF_TRY(od.fac32.ensure(al, (size_t)len * 4));
  return {};
}

Status build_split_fac(OperatorData& od, hipStream_t s) {
  WF_HIP(launch_split_fac(od.g.n, od.lam64.as<double>(), (double)od.g.m, od.fac64.as<double>(),
                          od.fac32.as<float>(), s));
  od.fac_ready = true;
  return {};
}

Status ensure_split_fac(const Allocator& al, OperatorData& od, hipStream_t s) {
  if (od.fac_ready) return {};
  WF_TRY(alloc_split_fac(al, od));
  return build_split_fac(od, s);
}

template <typename T> static const T* fac_of(const OperatorData& od) {
  if constexpr (sizeof(T) == 8) return od.fac64.as<T>();
  else return od.fac32.as<T>();
}

// x pass from `in` to `out` (both half spectra), aux and b at out's positions
template <typename T>
static StrArgs<T> split_x_args(const OperatorData& od, const cplx<T>* in, cplx<T>* out,
                               const cplx<T>* aux, const cplx<double>* bvec, const CgState* st,
                               int skip, double* partials) {
  const Grid& g = od.g;
  const int tb = strided_tb(g.n, sizeof(T) == 8);
  StrArgs<T> a{};
  a.s0 = seg_x_main<T>(out, g, tb);
  a.s1 = seg_x_nyq<T>(out + g.spec_main, g, tb);
  a.s0.in = in;
  a.s1.in = in + g.spec_main;
  a.s0.aux = aux;
  a.s1.aux = aux ? aux + g.spec_main : nullptr;
  a.s0.bvec = bvec;
  a.s1.bvec = bvec ? bvec + g.spec_main : nullptr;
  a.nblk0 = a.s0.n_outer * a.s0.n_btiles;
  a.nblk1 = a.s1.n_outer * a.s1.n_btiles;
  a.tw = tw_of<T>(od);
  a.st = skip != SKIP_NONE ? st : nullptr;
  a.skip = skip;
  a.fac = fac_of<T>(od);
  a.rhs_fac = od.rhs_fac;
  a.in_scale = 1.0 / (double)g.m;
  a.partials = partials;
  return a;
}

template <typename T>
Status split_passes(const OperatorData& od, int mode, const T* pin, cplx<T>* work, T* out,
                    const double* bh, CgState* st, double* partials, int nrhs, int skip,
                    hipStream_t s, const T* rdir, T* xdir) {
  const Grid& g = od.g;
  const bool f64 = sizeof(T) == 8;
  const double vb = (double)sizeof(T) * g.m * nrhs;
  const double sb = 2.0 * sizeof(T) * g.spec_total * nrhs;
  // each x pass reads the factor table once (per RHS when each has its own)
  const double fb = (double)sizeof(T) * split_fac_elems(g.n) * (od.rhs_fac ? nrhs : 1);
  const cplx<T>* pc = reinterpret_cast<const cplx<T>*>(pin);
  // the folded iteration (FWD_CGQF with rdir): the x inverse's partials (r.r,
  // p.p) at the start of `partials`, then per RHS the z middle pass's sums
  // (nzb) and the x forward's (2 nxb)
  const bool fold = rdir && mode == SM_FWD_CGQF;
  const int nzb = zpass_blocks(g.n, g.nrows, f64);
  double* part_z = partials;
  double* part_x = partials;
  if (fold) {
    const StrArgs<T> probe = split_x_args<T>(od, nullptr, work, nullptr, nullptr, st, skip, nullptr);
    const int64_t nxb = probe.nblk0 + probe.nblk1;
    if (nzb + 2 * nxb > partials_per_rhs(g)) return fail(WF_EINVAL, "partials too small");
    part_x = partials + (int64_t)nrhs * nzb;
  }
  if (fold) {
    // folded CG: r, q', p, x in; r, p, x and the x-transformed work spectrum
    // out; then the new r.r and p.p
    StrArgs<T> xa = split_x_args<T>(od, reinterpret_cast<const cplx<T>*>(rdir), work, nullptr,
                                    nullptr, st, skip, partials);
    xa.s0.p = const_cast<cplx<T>*>(pc);
    xa.s1.p = xa.s0.p + g.spec_main;
    xa.s0.x = reinterpret_cast<cplx<T>*>(xdir);
    xa.s1.x = xa.s0.x + g.spec_main;
    xa.s0.r = const_cast<cplx<T>*>(reinterpret_cast<const cplx<T>*>(rdir));
    xa.s1.r = xa.s0.r + g.spec_main;
    xa.s0.q = reinterpret_cast<const cplx<T>*>(out);
    xa.s1.q = xa.s0.q + g.spec_main;
    {
      ProfScope ps(od.prof, f64 ? WF_PROF_SXINV_F64 : WF_PROF_SXINV_F32, 8 * sb + fb, s);
      WF_HIP(launch_strided<T>(g.n, SM_INV_FOLD, xa, nrhs, s));
    }
    WF_HIP(launch_finalize(FIN_RRF, partials, xa.nblk0 + xa.nblk1, skip, st, nrhs, s));
  } else if (rdir) {
    // CG: r, p, x in; p, x and the x-transformed work spectrum out
    ProfScope ps(od.prof, f64 ? WF_PROF_SXINV_F64 : WF_PROF_SXINV_F32, 6 * sb + fb, s);
    StrArgs<T> xa = split_x_args<T>(od, reinterpret_cast<const cplx<T>*>(rdir), work, nullptr,
                                    nullptr, st, skip, nullptr);
    xa.s0.p = const_cast<cplx<T>*>(pc);
    xa.s1.p = xa.s0.p + g.spec_main;
    xa.s0.x = reinterpret_cast<cplx<T>*>(xdir);
    xa.s1.x = xa.s0.x + g.spec_main;
    WF_HIP(launch_strided<T>(g.n, SM_INV_DIR, xa, nrhs, s));
  } else {
    // p in, scaled and transformed along x into the work spectrum
    ProfScope ps(od.prof, f64 ? WF_PROF_SXINV_F64 : WF_PROF_SXINV_F32, 2 * sb + fb, s);
    WF_HIP(launch_strided<T>(g.n, SM_INV_SCALE,
                             split_x_args<T>(od, pc, work, nullptr, nullptr, st, skip, nullptr),
                             nrhs, s));
  }
  {
    ProfScope ps(od.prof, f64 ? WF_PROF_YINV_F64 : WF_PROF_YINV_F32, 2 * sb, s);
    WF_HIP(launch_strided<T>(g.n, SM_INV, str_args<T>(od, work, false, st, skip), nrhs, s));
  }
  {
    ZmidArgs<T> zm{};
    zm.spec_main = work;
    zm.spec_nyq = work + g.spec_main;
    zm.rhs_main = g.spec_total;
    zm.rhs_nyq = g.spec_total;
    set_noise_diag<T>(od, zm);
    zm.tw = tw_of<T>(od);
    zm.st = st;
    zm.skip = skip;
    zm.partials = fold ? part_z : nullptr;
    // spectrum in and out (in place), the noise diagonal in (once for all RHS
    // unless SD)
    ProfScope ps(od.prof, f64 ? WF_PROF_SZW_F64 : WF_PROF_SZW_F32,
                 2 * sb + (double)sizeof(T) * g.m * (od.sd ? nrhs : 1), s);
    WF_HIP(launch_zmid<T>(g.n, zm, g.nrows, nrhs, s));
  }
  {
    ProfScope ps(od.prof, f64 ? WF_PROF_YFWD_F64 : WF_PROF_YFWD_F32, 2 * sb, s);
    WF_HIP(launch_strided<T>(g.n, SM_FWD, str_args<T>(od, work, false, st, skip), nrhs, s));
  }
  const StrArgs<T> xa = split_x_args<T>(od, work, reinterpret_cast<cplx<T>*>(out), pc,
                                        reinterpret_cast<const cplx<double>*>(bh), st, skip,
                                        fold ? part_x : partials);
  {
    // work spectrum in, result out; CGQ also reads p, RES y and b (FP64); the
    // folded iteration's CGQF reads p at the monopole only
    double xb = 2 * sb + fb;
    if (mode == SM_FWD_CGQ) xb += sb;
    if (mode == SM_FWD_RES) xb += 2 * sb;
    ProfScope ps(od.prof, f64 ? WF_PROF_SXFWD_F64 : WF_PROF_SXFWD_F32, xb, s);
    WF_HIP(launch_strided<T>(g.n, mode, xa, nrhs, s));
  }
  const int nxb = xa.nblk0 + xa.nblk1;
  if (fold)
    WF_HIP(launch_finalize_fold_pq(part_z, nzb, part_x, nxb, (double)g.m, skip, st, nrhs, s));
  else if (mode == SM_FWD_CGQ || mode == SM_FWD_RES)
    WF_HIP(launch_finalize(mode == SM_FWD_CGQ ? FIN_PQ : FIN_RES, partials, nxb, skip, st, nrhs, s));
  return {};
}
template Status split_passes<float>(const OperatorData&, int, const float*, cplx<float>*, float*,
                                    const double*, CgState*, double*, int, int, hipStream_t,
                                    const float*, float*);
template Status split_passes<double>(const OperatorData&, int, const double*, cplx<double>*,
                                     double*, const double*, CgState*, double*, int, int,
                                     hipStream_t, const double*, double*);

// b_hat = c sqrt(D) F b (FP64, one RHS after another share the launches)
Status split_rhs(const OperatorData& od, const double* b, cplx<double>* work, double* bh,
                 int nrhs, hipStream_t s) {
  const Grid& g = od.g;
  ZfwdArgs<double> zf{};
  zf.in = b;
  zf.out_main = work;
  zf.out_nyq = work + g.spec_main;
  zf.nkz_out = g.n / 2;
  zf.rhs_in = g.m;
  zf.rhs_main = g.spec_total;
  zf.rhs_nyq = g.spec_total;
  zf.tw = tw_of<double>(od);
  WF_HIP(launch_zfwd<double>(g.n, ZIN_REAL, zf, g.nrows, nrhs, s));
  WF_HIP(launch_strided<double>(g.n, SM_FWD, str_args<double>(od, work, false, nullptr, SKIP_NONE),
                                nrhs, s));
  WF_HIP(launch_strided<double>(g.n, SM_FWD_SCALE,
                                split_x_args<double>(od, work, reinterpret_cast<cplx<double>*>(bh),
                                                     nullptr, nullptr, nullptr, SKIP_NONE, nullptr),
                                nrhs, s));
  return {};
}

// s = C y from the half-spectrum y (FP64): scaled x inverse, y inverse, z to real
Status split_solution(const OperatorData& od, const double* yh, cplx<double>* work, double* s_out,
                      int nrhs, hipStream_t s) {
  const Grid& g = od.g;
  WF_HIP(launch_strided<double>(
      g.n, SM_INV_SCALE,
      split_x_args<double>(od, reinterpret_cast<const cplx<double>*>(yh), work, nullptr, nullptr,
                           nullptr, SKIP_NONE, nullptr),
      nrhs, s));
  WF_HIP(launch_strided<double>(g.n, SM_INV, str_args<double>(od, work, false, nullptr, SKIP_NONE),
                                nrhs, s));
  ZinvArgs<double> zi{};
  zi.in_main = work;
  zi.in_nyq = work + g.spec_main;
  zi.rhs_main = g.spec_total;
  zi.rhs_nyq = g.spec_total;
  zi.out = s_out;
  zi.rhs_out = g.m;
  zi.scale = 1.0;
  zi.tw = tw_of<double>(od);
  WF_HIP(launch_zinv<double>(g.n, ZOUT_REAL, zi, g.nrows, nrhs, s));
  return {};
}

template <typename T>
Status forward_passes(const OperatorData& od, const T* in, cplx<T>* spec, hipStream_t s) {
  const Grid& g = od.g;
  ZfwdArgs<T> zf{};
  zf.in = in;
  zf.out_main = spec;
  zf.out_nyq = spec + g.spec_main;
  zf.nkz_out = g.n / 2;
  zf.rhs_in = g.m;
  zf.rhs_main = g.spec_total;
  zf.rhs_nyq = g.spec_total;
  zf.tw = tw_of<T>(od);
  WF_HIP(launch_zfwd<T>(g.n, ZIN_REAL, zf, g.nrows, 1, s));
  WF_HIP(launch_strided<T>(g.n, SM_FWD, str_args<T>(od, spec, false, nullptr, SKIP_NONE), 1, s));
  WF_HIP(launch_strided<T>(g.n, SM_FWD, str_args<T>(od, spec, true, nullptr, SKIP_NONE), 1, s));
  return {};
}
template Status forward_passes<float>(const OperatorData&, const float*, cplx<float>*, hipStream_t);
template Status forward_passes<double>(const OperatorData&, const double*, cplx<double>*,
                                       hipStream_t);

// ---------------------------------------------------------------------------
// gridding: deposit, then (s = 2) low-pass and resample (Sec. 3.1.2)
// ---------------------------------------------------------------------------
Status run_deposit(const Allocator& al, const OperatorData& od, DepositWork& dw,
                   const double* xyz, int64_t ngal, int scheme, int ss, double* nobs,
                   hipStream_t s) {
  const Grid& g = od.g;
  const int n = g.n, nf = ss * n;
  const int64_t mf = (int64_t)nf * nf * nf;
  WF_TRY(dw.grid.ensure(al, (size_t)mf * 8));
  long long* grid = dw.grid.as<long long>();
  const double c = (double)nf / g.box;
  {
    const int st = scheme == WF_NGP ? 1 : (scheme == WF_CIC ? 8 : 27);
    ProfScope ps(od.prof, WF_PROF_DEPOSIT, 8.0 * mf + 24.0 * ngal + 16.0 * st * ngal, s, true);
    WF_HIP(launch_fill_i64(grid, mf, s));
    WF_HIP(launch_deposit(scheme, xyz, ngal, c, nf, grid, s));
  }
  const double unit = scheme == WF_NGP ? 1.0 : std::ldexp(1.0, -39);
  return run_lowpass(al, od, dw, grid, nullptr, unit, ss, nobs, s);
}

Status run_lowpass(const Allocator& al, const OperatorData& od, DepositWork& dw,
                   const long long* grid, const double* dgrid, double unit, int ss, double* nobs,
                   hipStream_t s) {
  const Grid& g = od.g;
  const int n = g.n, nf = ss * n;
  const int64_t mf = (int64_t)nf * nf * nf;
  if (ss == 1) {
    if (grid) WF_HIP(launch_i64_to_f64(nobs, grid, unit, g.m, s));
    else WF_HIP(hipMemcpyAsync(nobs, dgrid, (size_t)g.m * 8, hipMemcpyDeviceToDevice, s));
    return {};
  }
  // fine forward transform, keeping kz < n/2
  const int h = n / 2;
  ProfScope pss(od.prof, WF_PROF_SUPERSAMPLE,
                8.0 * mf + 2 * 16.0 * nf * nf * h + 2 * 16.0 * nf * n * h + 16.0 * g.spec_total * 5 +
                    8.0 * g.m,
                s, true);
  if (dw.tw_fine_n != nf) {
    WF_TRY(make_twiddles(al, nf, dw.tw_fine, nullptr, s));
    dw.tw_fine_n = nf;
  }
  const int64_t fine_spec = (int64_t)nf * nf * h;
  WF_TRY(dw.fine_spec.ensure(al, (size_t)fine_spec * 16));
  auto* fs = dw.fine_spec.as<double2>();
  const auto* twf = dw.tw_fine.as<double2>();
  ZfwdArgs<double> zf{};
  zf.gin = grid;
  zf.in = dgrid;
  zf.unit = unit;
  zf.out_main = fs;
  zf.out_nyq = nullptr;
  zf.nkz_out = h;
  zf.tw = twf;
  WF_HIP(launch_zfwd<double>(nf, grid ? ZIN_I64 : ZIN_REAL, zf, (int64_t)nf * nf, 1, s));

  // y: fine [nf x][nf y][h] -> [nf x][n y][h], keeping |m_y| < n/2
  const int tbf = strided_tb(nf, true);
  const int64_t ysz = (int64_t)nf * n * h;
  WF_TRY(dw.spec_y.ensure(al, (size_t)ysz * 16));
  auto* sy = dw.spec_y.as<double2>();
  {
    StrArgs<double> a{};
    Seg<double>& q = a.s0;
    q.in = fs;
    q.out = sy;
    q.in_outer = (int64_t)nf * h;
    q.in_axis = h;
    q.in_batch = 1;
    q.out_outer = (int64_t)n * h;
    q.out_axis = h;
    q.out_batch = 1;
    q.n_outer = nf;
    q.n_btiles = h / tbf;
    q.n_out = n;
    a.nblk0 = q.n_outer * q.n_btiles;
    a.nblk1 = 0;
    a.tw = twf;
    WF_HIP(launch_strided<double>(nf, SM_FWD_CROP, a, 1, s));
  }
  // x: [nf x][n y][h] -> coarse main [n x][n y][h], keeping |m_x| < n/2
  WF_TRY(dw.spec_c.ensure(al, (size_t)g.spec_total * 16));
  auto* sc = dw.spec_c.as<double2>();
  {
    StrArgs<double> a{};
    Seg<double>& q = a.s0;
    q.in = sy;
    q.out = sc;
    q.in_outer = h;
    q.in_axis = (int64_t)n * h;
    q.in_batch = 1;
    q.out_outer = h;
    q.out_axis = (int64_t)n * h;
    q.out_batch = 1;
    q.n_outer = n;
    q.n_btiles = h / tbf;
    q.n_out = n;
    a.nblk0 = q.n_outer * q.n_btiles;
    a.nblk1 = 0;
    a.tw = twf;
    WF_HIP(launch_strided<double>(nf, SM_FWD_CROP, a, 1, s));
  }
  // the target Nyquist planes are dropped
  WF_HIP(launch_fill_c64(sc + g.spec_main, (int64_t)n * n, s));
  // coarse inverse: x, y, then z to real with 1/n^3
  WF_HIP(launch_strided<double>(n, SM_INV, str_args<double>(od, sc, true, nullptr, SKIP_NONE), 1, s));
  WF_HIP(launch_strided<double>(n, SM_INV, str_args<double>(od, sc, false, nullptr, SKIP_NONE), 1, s));
  ZinvArgs<double> zi{};
  zi.in_main = sc;
  zi.in_nyq = sc + g.spec_main;
  zi.out = nobs;
  zi.scale = 1.0 / (double)g.m;
  zi.tw = od.tw64.as<double2>();
  WF_HIP(launch_zinv<double>(n, ZOUT_REAL, zi, g.nrows, 1, s));
  return {};
}

// Bytes per cell of one CG iteration.  Plain form, FP32: 76 (FP64 doubles
// it).  Split form, FP64: 152, a half spectrum being 8 B per cell: x inverse
// with the direction update 48 (r, p, x in; p, x, work out), y 16, z middle
// 24, y 16, x forward with q 24, r update 24.  Split form, FP32 (the folded
// iteration): 68 -- x inverse with the r update and the direction 32 (r, q',
// p, x in; r, p, x, work out), y 8, z middle 12, y 8, x forward with q' 8
// (work in, q' out).  The split x passes also read the factor table once.
double model_bytes_iteration(bool fp64, bool split) {
  if (fp64) return 152.0;
  return split ? 68.0 : 76.0;
}
// FP64 residual b - A x, also 104 in both forms (split: x inverse 16, y 16,
// z middle 24, y 16, x forward with y and b in 32)
double model_bytes_residual(bool /*split*/) { return 104.0; }

}  // namespace wf
