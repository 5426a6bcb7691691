// Host-side internals shared by the context API, the batch driver and the
// server.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/wiener.h"
#include "launch.h"

namespace wf {

struct Status {
  wf_status code = WF_OK;
  std::string msg;
  bool ok() const { return code == WF_OK; }
};

inline Status fail(wf_status c, std::string m) { return Status{c, std::move(m)}; }
inline Status hip_fail(hipError_t e, const char* what) {
  return Status{WF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

#define WF_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)
#define WF_TRY(expr)            \
  do {                          \
    Status s_ = (expr);         \
    if (!s_.ok()) return s_;    \
  } while (0)

// Device allocator: caller callbacks or hipMalloc.
struct Allocator {
  wf_alloc_fn alloc = nullptr;
  wf_free_fn free_fn = nullptr;
  void* user = nullptr;
  int device = 0;
  void* get(size_t bytes) const;
  void put(void* p) const;
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  const Allocator* a = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();
  Status ensure(const Allocator& al, size_t b);  // keeps contents only if big enough already
  // non-owning alias of memory owned elsewhere (never freed through this buffer)
  void alias(void* ptr, size_t b) {
    release();
    p = ptr;
    bytes = b;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Live kernel timing with HIP events, harvested at synchronisation points.
// A bracket of one launch hands its events to that launch, which the runtime
// stamps with the dispatch's own start and end; a bracket of several launches
// records the events around them as markers (without the system-scope fence,
// a cache writeback at each record).  With every > 1 only one bracket in
// `every` of each class is timed.
struct Profiler {
  bool on = false;
  int every = 1;
  int64_t seen[WF_PROF_KINDS] = {};
  struct Pair {
    hipEvent_t a, b;
    int kind;
    double bytes;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pair> pending;
  std::vector<float> dur[WF_PROF_KINDS];     // ms of every harvested launch
  std::vector<double> byt[WF_PROF_KINDS];
  // Totals over full-work launches: a launch shorter than 0.8 of its class's
  // median did less (right-hand sides already stopped, or a first direction
  // that reads fewer vectors) and is counted as skipped.
  void totals(int64_t* launches, int64_t* skipped, double* ms, double* bytes) const;
  ~Profiler();
  void clear();
  int begin(int kind, double bytes, hipStream_t s, bool multi);
  void end(int idx, hipStream_t s, bool multi);
  void harvest();   // all recorded events must have completed
};

// RAII bracket of one launch.
struct ProfScope {
  Profiler* p;
  hipStream_t s;
  bool multi;
  int idx;
  // multi: the bracket holds more than one launch
  ProfScope(Profiler* p_, int kind, double bytes, hipStream_t s_, bool multi_ = false)
      : p(p_), s(s_), multi(multi_), idx(p_ ? p_->begin(kind, bytes, s_, multi_) : -1) {}
  ~ProfScope() {
    if (p && idx >= 0) p->end(idx, s, multi);
  }
};

// Geometry of one n^3 grid and its half spectrum layout.
struct Grid {
  int n = 0;
  double box = 0.0;
  int64_t m = 0;        // n^3
  int64_t nrows = 0;    // n^2
  int64_t spec_main = 0;  // n * n * n/2 complex
  int64_t spec_total = 0; // + n * n (Nyquist plane)
  int64_t lamlen = 0;   // 3 (n/2)^2 + 1
  int64_t xlamlen = 0;  // elements of the x-pass Lambda rows
  void set(int n_, double box_);
};

// The operator's constant data on the device (shared by every RHS of a grid).
struct OperatorData {
  Grid g;
  DevBuf w64, w32, tw64, tw32;
  DevBuf lam64;           // Lambda over |m|^2 (FP64)
  DevBuf xlam64, xlam32;  // the same, expanded into the x-pass rows
  DevBuf fac64, fac32;    // prior-split factor c over (|my|, |mx|, kz), built on demand
  bool fac_ready = false;
  // signal-dependent noise: while sd is set the operator's noise diagonal is
  // dg (nbar w g per RHS, n^3 apart) instead of nbar w
  bool sd = false;
  DevBuf dg64, dg32;
  // per-RHS tables (several solves of one grid with their own masks and
  // priors): element strides between the RHS's copies, 0 when shared
  int64_t rhs_w = 0, rhs_lam = 0, rhs_xlam = 0, rhs_fac = 0;
  Profiler* prof = nullptr;   // optional
  // a one-RHS view of RHS `slot` of `src` (tables of that RHS, shared
  // twiddles, box `box`); the view owns nothing
  void make_view(const OperatorData& src, int slot, double box);
};

// Workspace of solves on a grid for `nrhs` right-hand sides.
struct SolveWork {
  int nrhs = 0;
  // prior-split solves: x, r, p, q hold half spectra (vlen = 2 spec_total
  // elements per RHS, complex interleaved) and x64 receives the real solution
  // (n^3 per RHS) at the end; otherwise vlen = n^3
  bool split = false;
  int64_t vlen = 0;
  DevBuf b64, x64, r64, p64, q64, spec64;
  DevBuf x32, r32, p32, q32, spec32;
  DevBuf bh64, u64;  // split: C b (half spectrum), a real field per RHS
  DevBuf state, partials;
  CgState* st_host = nullptr;   // pinned mirror of the state array
  int st_cap = 0;
  bool view = false;            // a view of one RHS of another SolveWork (owns nothing)
  ~SolveWork();
  // one-RHS view of RHS `slot` of src (its vectors, state and mirror; the
  // partials of src are shared, so the view's launches must not overlap
  // src's)
  void make_view(const SolveWork& src, const Grid& g, int slot);
  // b, x, r and the FP64 spectrum always; p, q (FP64 CG); the FP32 set (mixed)
  Status ensure(const Allocator& al, const Grid& g, int nrhs, bool fp64_cg, bool mixed,
                bool split = false);
  Status pull_state(hipStream_t s);
};

// doubles of block partials a solve keeps per RHS
int64_t partials_per_rhs(const Grid& g);
Status make_twiddles(const Allocator& al, int n, DevBuf& tw64, DevBuf* tw32, hipStream_t s);
// Prior-split operator (C A C) on half-spectrum vectors (stride spec_total
// complex per RHS).  ensure_split_fac builds c once per power spectrum.
// split_passes: q = C A C p (mode SM_FWD_CGQ, with p.q and FIN_PQ) or
// r = b_hat - C A C y (SM_FWD_RES, FP64, with ||r||^2 and FIN_RES), through
// the half spectrum `work`.  With rdir (and xdir) the CG direction update
// p = r + beta p (and the pending x += alpha p) happens in the first pass.  split_rhs: b_hat = C b.  split_solution: s = C y
// into real fields.
Status ensure_split_fac(const Allocator& al, OperatorData& od, hipStream_t s);
Status alloc_split_fac(const Allocator& al, OperatorData& od);
Status build_split_fac(OperatorData& od, hipStream_t s);
template <typename T>
Status split_passes(const OperatorData& od, int mode, const T* pin, cplx<T>* work, T* out,
                    const double* bh, CgState* st, double* partials, int nrhs, int skip,
                    hipStream_t s, const T* rdir = nullptr, T* xdir = nullptr);
Status split_rhs(const OperatorData& od, const double* b, cplx<double>* work, double* bh,
                 int nrhs, hipStream_t s);
Status split_solution(const OperatorData& od, const double* yh, cplx<double>* work, double* s_out,
                      int nrhs, hipStream_t s);
// x-pass Lambda rows: allocation, and expansion from lam64 (on stream s)
Status alloc_xlam(const Allocator& al, OperatorData& od);
Status build_xlam(OperatorData& od, hipStream_t s);
Status upload(void* dst, const void* src, size_t bytes, wf_mem mem, hipStream_t s);
Status download(void* dst, const void* src, size_t bytes, wf_mem mem, hipStream_t s);

// Operator pipeline (five sweeps) on `nrhs` vectors laid out with stride g.m.
template <typename T>
Status operator_passes(const OperatorData& od, int zin_mode, const T* in_or_r, T* p, T* x,
                       cplx<T>* spec, int zout_mode, T* out, const T* aux,
                       const double* bvec, CgState* st, double* partials, int nrhs,
                       int skip, hipStream_t s);

// Forward transform only (test hook): z, y, x forward passes.
template <typename T>
Status forward_passes(const OperatorData& od, const T* in, cplx<T>* spec, hipStream_t s);

// Gridding of one catalogue into n_obs (n^3 doubles) -- Sec. 3.1.2.
struct DepositWork {
  DevBuf grid, fine_spec, spec_y, spec_c, tw_fine, flag;
  int tw_fine_n = 0;  // length tw_fine holds the twiddles of
};
// The low-pass and resampling of a deposit grid (int64 units, or FP64 when
// `grid` is null) into the target-grid n_obs (Sec. 3.1.2).
Status run_lowpass(const Allocator& al, const OperatorData& od, DepositWork& dw,
                   const long long* grid, const double* dgrid, double unit, int ss, double* nobs,
                   hipStream_t s);
template <typename T> StrArgs<T> spectrum_args(const OperatorData& od, cplx<T>* spec, bool xpass);
// post-processing (post.hip)
hipError_t launch_rsd_factor(double dk2, double beta, double sigma, double* out, int64_t len,
                             hipStream_t s);
hipError_t launch_filter_table(int kind, double dk2, double a, double b, double c,
                               const double* table, int64_t len, double scale, double* out,
                               int* flag, hipStream_t s);
Status filter_passes(const OperatorData& od, const double* hrows, const double* in,
                     cplx<double>* spec, double* out, hipStream_t s);
Status field_sums(const double* v, const double* w, int64_t m, DevBuf& parts, const Allocator& al,
                  double out[5], hipStream_t s);
// field_sums with its partials in a static device array (no allocation);
// `device` must be the current device
Status field_sums_noalloc(const double* v, const double* w, int64_t m, int device, double out[5],
                          hipStream_t s);
// count, mean, variance, skewness, excess kurtosis from the sums of 1, v .. v^4
void moments_from_sums(const double sm[5], double out5[5]);
Status compare_sums(const double* rec, const double* tru, const double* w, int64_t m, DevBuf& parts,
                    DevBuf& flag, const Allocator& al, double out[6], bool* kl_ok, hipStream_t s);
hipError_t launch_deposit_iw(int scheme, const double* xyz, int64_t ngal, double c, int nd,
                             double ct, int n, const double* w, double* grid, int* flag,
                             hipStream_t s);
hipError_t launch_overdensity(double* v, int64_t m, double inv_nbar, hipStream_t s);
Status run_deposit(const Allocator& al, const OperatorData& od, DepositWork& dw,
                   const double* xyz_dev, int64_t ngal, int scheme, int supersample,
                   double* nobs_dev, hipStream_t s);

// Algorithmic HBM bytes of one CG iteration (model of the five sweeps plus
// the vector update) and of one FP64 residual recomputation, per cell.
double model_bytes_iteration(bool fp64, bool split = false);
double model_bytes_residual(bool split = false);

}  // namespace wf
