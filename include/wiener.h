/*
 * wiener.h -- C ABI of the MI355X Wiener-reconstruction library.
 *
 * The library computes the mean of the Wiener filter in its signal-space form
 * (eq:WF, Sec. 3.3.1 of Kitaura et al., "Cosmic cartography of the large-scale
 * structure with SDSS DR6"):
 *
 *     s = (S^-1 + W^T N^-1 W)^-1 W^T N^-1 delta^o
 *
 * on a periodic n^3 grid of side L, with
 *   - W = diag(w), the 3D completeness (Sec. 3.1.3; response of eq:RO with no
 *     bias or redshift-space operator),
 *   - N = diag(w / nbar), the LSQ shot-noise covariance (eq:noiseav),
 *   - delta^o = n^o / nbar - w, the observed overdensity (eq:datamodel), with
 *     nbar = N_gal / sum(w) (eq:nmean, per cell),
 *   - S diagonal in Fourier space with eigenvalues P(k)/dV (Sec. 3.3.1),
 *   - n^o the galaxy field gridded by mass assignment on the comb of
 *     def:ngrid (Sec. 3.1.2), optionally 2x supersampled and low-passed.
 * Multiplying by nbar, the library solves the SPD system
 *
 *     A s = b,  A = F^-1 diag(Lambda) F + diag(nbar w),
 *     Lambda_m = dV / P(k_m) (m != 0), Lambda_0 = 0,
 *     b = n^o - nbar w on cells with w > 0, 0 elsewhere,
 *
 * by conjugate gradients (the "iterative Krylov-space inversion" of Sec. 1),
 * in FP64 or in mixed precision (FP32 operator inside an FP64 iterative
 * refinement loop).
 *
 * Conventions (all entry points):
 *   - Every call returns a wf_status.  wf_last_error() gives a message for the
 *     most recent failing call on that context.  No exception or abort crosses
 *     the ABI.
 *   - Grid arrays are C-order [x][y][z] with z contiguous, n^3 doubles; grid
 *     nodes sit at x = i * L / n, i in [0, n).
 *   - A pointer argument carries a wf_mem tag saying whether it is host memory
 *     or device memory on the context's GPU.  With WF_HOST the call has
 *     finished using the buffer when it returns.  With WF_DEVICE the work is
 *     ordered on the context's stream (results are valid once that stream has
 *     reached the call) -- except where a call documents that it synchronises.
 *   - The library never keeps a caller pointer after a call returns; inputs are
 *     copied.  Outputs are written only on WF_OK (and for WF_ENOTCONV, see
 *     wf_solve).  Device memory is obtained through the allocator callbacks
 *     given at context creation (NULL callbacks: hipMalloc / hipFree).
 *   - One context per host thread at a time.  Different contexts are
 *     independent.
 */
#ifndef WIENER_H
#define WIENER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WF_ABI_VERSION 3

typedef enum {
  WF_OK = 0,
  WF_EINVAL = 1,      /* an argument is out of range, non-finite or malformed */
  WF_ESTATE = 2,      /* calls made out of order (e.g. solve before data)     */
  WF_ENOMEM = 3,      /* device allocation failed / footprint over budget     */
  WF_EDEVICE = 4,     /* a HIP runtime call failed                            */
  WF_ENOTCONV = 5,    /* max_iter reached before the tolerance                */
  WF_EOVERFLOW = 6,   /* too many galaxies for exact integer accumulation     */
  WF_EBREAKDOWN = 7   /* p.Ap <= 0 or non-finite: operator not SPD            */
} wf_status;

typedef enum { WF_HOST = 0, WF_DEVICE = 1 } wf_mem;

/* Mass-assignment kernels named in Sec. 3.1.2. */
typedef enum { WF_NGP = 0, WF_CIC = 1, WF_TSC = 2 } wf_scheme;

typedef enum {
  WF_FP64 = 0,   /* FP64 vectors, FFTs and reductions                          */
  WF_MIXED = 1   /* FP32 operator and vectors, FP64 dots, FP64 residual
                    recomputation and solution (reliable-update refinement) */
} wf_precision;

/* Preconditioning of the CG.
 *   WF_PRECOND_NONE   plain CG on A s = b.
 *   WF_PRECOND_PRIOR  CG on the prior-split system (C A C) y = C b, s = C y,
 *                     with C = S^(1/2) the square root of the prior covariance
 *                     (Sec. 3.3.1: S is diagonal in Fourier space with
 *                     eigenvalues P/dV; C takes their square roots, the
 *                     monopole the |m|^2 = 1 value).  Same solution A^-1 b;
 *                     the spectrum of C A C lies within
 *                     [.., 1 + nbar max(w) max(P/dV)] at any resolution, while
 *                     that of A spans the whole range of dV/P.  The CG vectors
 *                     live in the half spectrum; tol applies to
 *                     ||C (b - A s)|| / ||C b||; rel_res_true still reports
 *                     ||b - A s|| / ||b|| (one FP64 operator application at
 *                     the end). */
typedef enum { WF_PRECOND_NONE = 0, WF_PRECOND_PRIOR = 1 } wf_precond;

/* Device allocator callbacks (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` on the context's device, aligned
 * to 256 bytes, or NULL. */
typedef void* (*wf_alloc_fn)(size_t bytes, void* user);
typedef void (*wf_free_fn)(void* dptr, void* user);

typedef struct wf_ctx wf_ctx;
typedef struct wf_server wf_server;

/* Solver options.
 *   tol         stop when ||b - A x|| / ||b|| <= tol.  FP64: on the recursive
 *               CG residual.  MIXED: on the residual recomputed with the FP64
 *               operator.  tol = 0 runs exactly max_iter iterations.
 *   max_iter    CG iterations (MIXED: FP32 iterations).
 *   inner_tol   MIXED only: reliable-update factor.  The FP32 correction is
 *               folded into the FP64 solution and the residual recomputed in
 *               FP64 each time the FP32 recursive residual has dropped by this
 *               factor since the previous recomputation (0: default 0.1).
 *   max_outer   MIXED only: maximum number of FP64 residual recomputations
 *               (0: no limit).
 *   check_every host convergence checks every this many iterations (0: 16).
 *               Results do not depend on it: the device stops iterating at
 *               convergence by itself.
 *   precond     wf_precond.
 *   err_tol     MIXED only (0: the default 5e-7; < 0: no such condition):
 *               once the FP64 residual meets tol the solve goes on through
 *               the reliable updates that reduce the residual by another
 *               factor of 10 (one at the default inner_tol), and stops at the
 *               first update, with tol met, after which their summed changes
 *               of the solution s are at most err_tol relative
 *               (||s_new - s_old|| / ||s_new||, on s = C y for the
 *               prior-split form).  The residual
 *               alone does not bound the error of a mixed solve: FP32 rounding
 *               of the operator, which grows with nbar, leaves large-scale
 *               error in the unobserved region that the residual barely
 *               weights until it has dropped further; that error shows in the
 *               change the following FP64 refresh makes.  An error that stays
 *               put between refreshes does not: at extreme densities in small
 *               caps (nbar ~ 800 in a 30 degree cap) a uniform offset of the
 *               unobserved volume of ~1e-6 can remain; FP64 has no such floor. */
typedef struct {
  wf_precision precision;
  double tol;
  int32_t max_iter;
  double inner_tol;
  int32_t max_outer;
  int32_t check_every;
  int32_t precond;
  double err_tol;
} wf_solve_opts;

typedef struct {
  int32_t iters_total;        /* CG iterations                                */
  int32_t outer_steps;        /* MIXED: FP64 residual recomputations          */
  double rel_res_recursive;   /* last recursive residual ||r|| / ||b||        */
  double rel_res_true;        /* ||b - A x|| / ||b|| with the FP64 operator   */
  double time_ms;             /* wall time of the solve on the device         */
  double model_bytes;         /* algorithmic HBM bytes moved by the solve     */
  double nbar;                /* mean density per cell used                   */
  int32_t status;             /* wf_status of the solve                       */
  double last_change;         /* MIXED: relative change of s made by the last
                                 reliable update (see err_tol): with err_tol,
                                 an estimate of the error left; 0 for FP64    */
  double latency_ms;          /* server: submit -> result ready on the host;
                                 0 elsewhere                                  */
  int32_t stagnated;          /* MIXED: 1 if the solve stopped (WF_ENOTCONV)
                                 because 4 reliable updates in a row did not
                                 bring its FP64 residual 10 % below the best
                                 so far: tol is below what the arithmetic
                                 reaches                                      */
} wf_solve_info;

/* ---- library ----------------------------------------------------------- */
int wf_abi_version(void);
const char* wf_status_str(wf_status s);

/* ---- context ----------------------------------------------------------- */
/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * owned by the caller (NULL: the null stream).  alloc/free may be NULL. */
wf_status wf_ctx_create(wf_ctx** out, int device, void* hip_stream,
                        wf_alloc_fn alloc, wf_free_fn free_fn, void* user);
wf_status wf_ctx_destroy(wf_ctx* ctx);
const char* wf_last_error(const wf_ctx* ctx);

/* Grid: n cells per axis, n = 2^a 3^b with b <= 1 and 8 <= n <= 512; box side
 * L > 0 in Mpc.  Resets every other input of the context. */
wf_status wf_set_grid(wf_ctx* ctx, int32_t n, double box_mpc);

/* 3D completeness w (Sec. 3.1.3, "w <= 1"): n^3 doubles, finite, 0 <= w <= 1,
 * not all zero; otherwise WF_EINVAL.  Synchronises. */
wf_status wf_set_mask(wf_ctx* ctx, const double* w, wf_mem mem);

/* Prior spectrum sampled on the |m|^2 lattice: p_by_m2[j] = P(k) in Mpc^3 at
 * k = 2 pi sqrt(j) / L, j = 0 .. 3 (n/2)^2 (len must equal that count).  Entry
 * 0 is ignored (Lambda_0 = 0); the others must be finite and > 0, else
 * WF_EINVAL.  Synchronises. */
wf_status wf_set_power(wf_ctx* ctx, const double* p_by_m2, int64_t len,
                       wf_mem mem);

/* Galaxy positions (Sec. 3.1.2 point-source field): xyz[n_gal][3] in Mpc with
 * 0 <= x < L on every axis (else WF_EINVAL); n_gal < 2^24 (else WF_EOVERFLOW,
 * the bound for exact int64 accumulation).  n_gal = 0 is allowed.
 * Synchronises. */
wf_status wf_set_galaxies(wf_ctx* ctx, const double* xyz, int64_t n_gal,
                          wf_mem mem);

/* Gridding (Sec. 3.1.2, def:ngrid): fixed-point mass assignment onto the
 * (supersample * n)^3 grid with exact int64 accumulation (weights in units of
 * 2^-39 for CIC/TSC, counts for NGP), then for supersample = 2 the ideal
 * low-pass (|m| < n/2 on every axis, Nyquist planes dropped) and resampling at
 * n^3; then nbar = N_gal / sum(w) and b.  Needs grid, mask and galaxies. */
wf_status wf_deposit(wf_ctx* ctx, wf_scheme scheme, int32_t supersample);

/* Copies out the last deposit: the integer (s n)^3 grid, n^o (n^3 doubles)
 * and nbar.  Any output may be NULL.  Synchronises. */
wf_status wf_get_deposit(wf_ctx* ctx, int64_t* fine_counts, double* n_obs,
                         double* nbar_cell, wf_mem mem);

/* Test hook: replaces the data vector by b (n^3) and nbar (> 0). */
wf_status wf_set_rhs(wf_ctx* ctx, const double* b, double nbar_cell,
                     wf_mem mem);

/* Test hook: Av = A v with the operator in the given precision (MIXED: the
 * FP32 operator on v rounded to FP32, result widened).  Needs grid, mask,
 * power and nbar (from wf_deposit or wf_set_rhs). */
wf_status wf_apply_operator(wf_ctx* ctx, wf_precision prec, const double* v,
                            double* Av, wf_mem mem);

/* Test hook: the unnormalised forward real-to-complex 3D DFT of v (n^3) in
 * numpy.fft.rfftn layout: spec[n][n][n/2+1] complex as interleaved doubles. */
wf_status wf_forward_spectrum(wf_ctx* ctx, wf_precision prec, const double* v,
                              double* spec, wf_mem mem);

/* Solves A s = b (see the top of this file) from s = 0 and writes s (n^3).
 * WF_ENOTCONV: tolerance not reached within max_iter; s_out holds the last
 * iterate and info is filled.  WF_EBREAKDOWN: s_out untouched.  info may be
 * NULL.  Synchronises. */
wf_status wf_solve(wf_ctx* ctx, const wf_solve_opts* opts, double* s_out,
                   wf_mem mem, wf_solve_info* info);

/* Krylov state of a solve (FP64 or mixed, plain or prior-split), for
 * checkpoint / resume.  wf_solve_begin starts a solve, wf_solve_step runs up
 * to `iters` more CG iterations (mixed: FP32 iterations, with the reliable
 * updates they call for), wf_solve_snapshot copies the state into host_buf of
 * wf_snapshot_bytes() bytes (the size for the active solve; without one, that
 * of a plain FP64 solve): the scalars and x, r, p in FP64, or for a mixed
 * solve the FP64 x and r and the FP32 x, r, p -- half spectra for the
 * prior-split form, whose FP32 iteration ends with its step pending until the
 * next iteration applies it and so also keeps q.  wf_solve_resume restores it into a context with the same
 * grid, mask, power and rhs (the snapshot records its form), and
 * wf_solve_finish writes s and info (a mixed solve stopped between reliable
 * updates first folds its FP32 correction and takes the FP64 residual, as an
 * update would).  Continuing from a snapshot gives bit-identical results,
 * equal to an uninterrupted wf_solve of as many iterations. */
wf_status wf_solve_begin(wf_ctx* ctx, const wf_solve_opts* opts);
wf_status wf_solve_step(wf_ctx* ctx, int32_t iters, int32_t* done);
size_t wf_snapshot_bytes(const wf_ctx* ctx);
wf_status wf_solve_snapshot(wf_ctx* ctx, void* host_buf, size_t bytes);
wf_status wf_solve_resume(wf_ctx* ctx, const void* host_buf, size_t bytes);
wf_status wf_solve_finish(wf_ctx* ctx, double* s_out, wf_mem mem,
                          wf_solve_info* info);

/* Multi-RHS solve: nrhs catalogues on the context's grid, mask and power,
 * each deposited (scheme, supersample) and solved in MIXED or FP64 precision
 * with batched kernels (one launch per pass covers every RHS).  xyz[i] holds
 * n_gal[i] galaxies (same rules as wf_set_galaxies); s_out[i] receives n^3
 * doubles; infos[i] (may be NULL) the per-RHS info.  Returns the worst status.
 * Synchronises. */
wf_status wf_solve_batch(wf_ctx* ctx, int32_t nrhs, const double* const* xyz,
                         const int64_t* n_gal, wf_scheme scheme,
                         int32_t supersample, const wf_solve_opts* opts,
                         double* const* s_out, wf_mem mem,
                         wf_solve_info* infos);

/* ---- signal-dependent noise (eq:noisecov, Sec. 3.4) -------------------- */
/* The SD formulation replaces the averaged noise w / nbar of each observed
 * cell by lambda^o / nbar^2, lambda^o estimating the expected observed count
 * w lambda.  The system solved is
 *   (F^-1 Lambda F + diag(nbar w g)) s = g (n^o - nbar w),  g = nbar w / lambda^o
 * on cells with w > 0 (cells with w = 0 carry no data and no noise term), with
 * n^o and nbar from the last wf_deposit.  Counts N are galaxies per nearest
 * target node (the NGP rule on the target grid).  Estimators:
 *   WF_NOISE_SD_MEAN       lambda^o = N^o + 1 (flat-prior mean, Sec. 3.4.1)
 *   WF_NOISE_SD_JACKKNIFE  lambda^o = w (N' + 1) / alpha, N' the counts of a
 *       binomial thinning that keeps each galaxy with probability alpha / w
 *       of its node (eq:selfunc; the + 1 keeps every observed cell's noise
 *       above zero).  Sample j of seed S keeps galaxy g when the first word of
 *       Philox4x32-10 (Salmon et al. 2011) with counter (g mod 2^32, g div
 *       2^32, j mod 2^32, 0) and key (S mod 2^32, S div 2^32) is below (alpha / w) 2^32
 *       (compared in double precision). */
typedef enum { WF_NOISE_SD_MEAN = 1, WF_NOISE_SD_JACKKNIFE = 2 } wf_noise;

/* Thinned counts N' of jackknife samples first .. first + count - 1 of the
 * context's galaxies: out holds count x n^3 int32 (sample-major, C order per
 * sample; only nodes with w > 0 count).  alpha in (0, w] at the node of every
 * galaxy, else WF_EINVAL.  Needs wf_set_grid, wf_set_mask, wf_set_galaxies.
 * Synchronises. */
wf_status wf_jackknife_counts(wf_ctx* ctx, double alpha, uint64_t seed, int64_t first,
                              int32_t count, int32_t* out, wf_mem mem);

/* SD Wiener reconstruction of the galaxies of the last wf_deposit (which must
 * follow the last wf_set_galaxies / wf_set_mask / wf_set_grid): nsamples
 * systems (1 for WF_NOISE_SD_MEAN; jackknife samples first .. first +
 * nsamples - 1), solved with the batched kernels in groups of up to 16 with
 * `opts`.  mean_out (n^3) receives the mean of the solutions (the paper's
 * jackknife estimate); samples_out (nsamples x n^3, may be NULL) each of them;
 * infos (nsamples, may be NULL) their infos.  Both outputs on `mem`.  Returns
 * the worst status (outputs written for WF_OK, WF_ENOTCONV and
 * WF_EBREAKDOWN).  alpha and seed are ignored by WF_NOISE_SD_MEAN.
 * Synchronises. */
wf_status wf_solve_sd(wf_ctx* ctx, const wf_solve_opts* opts, int32_t kind, double alpha,
                      uint64_t seed, int64_t first, int32_t nsamples, double* mean_out,
                      double* samples_out, wf_mem mem, wf_solve_info* infos);

/* ---- after the solve: redshift space, filters, comparators ------------- */
/* Redshift-distortion factor of Sec. 3.3.3: the angle average
 *   g(k) = <K D>_mu = int_0^1 (1 + beta mu^2)^2 / (1 + k^2 sigma^2 mu^2 / 2) dmu
 * of the Kaiser factor times the Lorentzian damping, at k = (2 pi / L) sqrt(j)
 * for j = 0 .. len - 1 (len <= 3 (n/2)^2 + 1; sigma in Mpc, e.g. the paper's
 * 500 km/s / H0).  P^s = g P^r is the redshift-space prior, to be passed to
 * wf_set_power.  Needs wf_set_grid.  Writes `out` (len doubles on `mem`). */
wf_status wf_rsd_factor(wf_ctx* ctx, double beta, double sigma_mpc, double* out,
                        int64_t len, wf_mem mem);

typedef enum {
  WF_FILTER_GAUSS = 0,       /* h = exp(-k^2 r_S^2 / 2): the Gaussian smoothing of
                                eq:GAUSS with radius a = r_S [Mpc] */
  WF_FILTER_RSD_DECONV = 1,  /* h = 1 / (b sqrt(g(k))): the deconvolution eq:DEC by
                                the angle-averaged redshift operator and a constant
                                bias, a = beta, b = sigma [Mpc], c = bias */
  WF_FILTER_TABLE = 2        /* h = table[j] at k = (2 pi / L) sqrt(j),
                                len = 3 (n/2)^2 + 1 */
} wf_filter_kind;

/* out = F^-1 diag(h(|k|)) F in on the context's grid (FP64, n^3 doubles each,
 * on `mem`; they may be the same buffer).  Non-finite h: WF_EINVAL. */
wf_status wf_fourier_filter(wf_ctx* ctx, int32_t kind, double a, double b, double c,
                            const double* table, int64_t len, const double* in,
                            double* out, wf_mem mem);

/* Moments of an n^3 field over all cells, or over those with w > 0
 * (masked != 0): out[0..4] = cell count, mean, variance, skewness, excess
 * kurtosis (population moments).  Synchronises. */
wf_status wf_field_moments(wf_ctx* ctx, const double* v, int32_t masked, double* out5,
                           wf_mem mem);

/* wf_field_moments for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same summation order, so the same bits, but the
 * block partials live in a static device array of 1024 x 5 + 8 doubles
 * (41 KB per GPU, held until the process ends) instead of a buffer from the
 * context's allocator; nothing is allocated.  v must be device memory on the
 * context's GPU (n^3 doubles; host memory: WF_EINVAL), out5 host memory.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (several threads, several contexts) race and must be serialised by the
 * caller.  Synchronises the context's stream. */
wf_status wf_field_moments_noalloc(wf_ctx* ctx, const double* v, int32_t masked, double* out5);

/* Quality measures of Sec. 4.1 between a reconstruction and a reference
 * field (n^3 each, over all cells or those with w > 0): out[0] = the
 * correlation coefficient r, out[1] = the Euclidean distance D_Euc,
 * out[2] = the Kullback-Leibler distance D_KL of 1 + delta (NaN where some
 * 1 + delta <= 0).  Synchronises. */
wf_status wf_compare_fields(wf_ctx* ctx, const double* rec, const double* truth,
                            int32_t masked, double* out3, wf_mem mem);

/* Inverse-weighting comparator (Sec. 4, the first step of the IW scheme):
 * every galaxy of wf_set_galaxies weighted by 1/w of its nearest target node,
 * deposited with `scheme` on the supersample-times-finer grid and low-passed
 * as in wf_deposit, then delta_IW = n_IW / nbar - 1 with nbar of eq:nmean.
 * A galaxy on a node with w = 0: WF_EINVAL.  FP64 atomic sums: reproducible to
 * rounding, not bit for bit.  Writes `out` (n^3 doubles on `mem`). */
wf_status wf_inverse_weighting(wf_ctx* ctx, wf_scheme scheme, int32_t supersample,
                               double* out, wf_mem mem);

/* ---- live kernel timing ------------------------------------------------ */
/* Kernel classes timed by the profiler: the five sweeps of one operator
 * application and the CG vector update, in FP32 (0..5) and FP64 (6..11),
 * then the gridding kernels; then the sweeps of the prior-split operator
 * that differ from those (its y passes, z forward pass and r update count
 * under the classes above): the direction update, the scaled x inverse pass,
 * the z inverse pass times nbar w, and the x forward pass that finishes
 * q = C A C p, in FP32 (14..17) and FP64 (18..21). */
#define WF_PROF_KINDS 22
typedef enum {
  WF_PROF_ZFWD_F32 = 0, WF_PROF_YFWD_F32, WF_PROF_XLAM_F32, WF_PROF_YINV_F32,
  WF_PROF_ZINV_F32, WF_PROF_UPDATE_F32,
  WF_PROF_ZFWD_F64, WF_PROF_YFWD_F64, WF_PROF_XLAM_F64, WF_PROF_YINV_F64,
  WF_PROF_ZINV_F64, WF_PROF_UPDATE_F64,
  WF_PROF_DEPOSIT, WF_PROF_SUPERSAMPLE,
  WF_PROF_SDIR_F32, WF_PROF_SXINV_F32, WF_PROF_SZW_F32, WF_PROF_SXFWD_F32,
  WF_PROF_SDIR_F64, WF_PROF_SXINV_F64, WF_PROF_SZW_F64, WF_PROF_SXFWD_F64
} wf_prof_kind;

/* Per class: full-work launches, their summed device time (HIP events that
 * the runtime stamps with each timed dispatch's start and end) and their
 * algorithmic HBM bytes (the bytes the pass must read and write once:
 * inputs, outputs, the half spectrum).  Launches that did less than the
 * class's full work (right-hand sides already stopped, or the first
 * direction of a CG cycle, which reads fewer vectors) run shorter than 0.8 of
 * the class's median: they are counted in `skipped` and left out of the
 * totals, whose bytes assume the full work. */
typedef struct {
  int64_t launches[WF_PROF_KINDS];
  int64_t skipped[WF_PROF_KINDS];
  double ms[WF_PROF_KINDS];
  double bytes[WF_PROF_KINDS];
} wf_profile;

/* Turns event timing off (0) or on and clears the counters: on = 1 times
   every launch, on = k > 1 one launch in k of each kernel class (the rest
   run without events, which keeps the timing's own cost off the work it
   measures).  Negative values are rejected with WF_EINVAL. */
wf_status wf_profile_enable(wf_ctx* ctx, int32_t on);
/* Synchronises the stream and returns the counters since enabling. */
wf_status wf_profile_read(wf_ctx* ctx, wf_profile* out);

/* Device bytes one solve needs at the peak of its phases (deposit or solve). */
size_t wf_footprint_bytes(int32_t n, int32_t supersample, wf_precision prec,
                          int32_t nrhs);

/* ---- serving ----------------------------------------------------------- */
/* A reconstruction request: all pointers are host memory, copied at submit. */
typedef struct {
  int32_t n;
  double box_mpc;
  const double* w;          /* n^3 */
  const double* p_by_m2;    /* 3 (n/2)^2 + 1 */
  const double* xyz;        /* [n_gal][3] */
  int64_t n_gal;
  wf_scheme scheme;
  int32_t supersample;
  wf_solve_opts opts;
} wf_request;

typedef struct {
  int64_t completed;
  int64_t failed;
  double solves_per_s;      /* completed / (last completion - first arrival) */
  double p50_ms, p99_ms;    /* submit -> result ready on the host            */
  size_t peak_bytes;        /* peak device bytes held by admitted requests   */
  int64_t cohorts;          /* batched solves started (see wf_server_create) */
  int32_t largest_cohort;   /* most requests in one batched solve            */
} wf_server_stats;

/* A continuous-batching server on one device.  Requests are admitted in
 * arrival order while their device memory fits in hbm_budget bytes and fewer
 * than max_active batched solves run: the request at the head of the queue is
 * admitted together with every queued request of equal grid, supersampling,
 * precision and preconditioning (up to 16, as many as fit; masks, priors,
 * boxes and catalogues may all differ) as one batched solve, whose every pass
 * is one launch for all of them.  Batched solves run concurrently on their
 * own streams (max_active of them).  With max_active > 1 the last free stream
 * only takes requests of grids up to 128^3 (the first such request in the
 * queue heads the batch), so small requests never wait behind large solves;
 * larger ones wait for another stream.  Krylov state stays on the device; a request's result
 * is copied out as soon as its own solve stops, and its gridding buffers are
 * returned as soon as its data vector is built.  A result is bitwise the same
 * whatever it was batched with.  wf_server_submit returns WF_ENOMEM if the
 * request can never fit. */
wf_status wf_server_create(wf_server** out, int device, size_t hbm_budget,
                           int32_t max_active, wf_alloc_fn alloc,
                           wf_free_fn free_fn, void* user);
wf_status wf_server_submit(wf_server* srv, const wf_request* req,
                           uint64_t* ticket);
/* done = 1 once the result is ready (info filled, may be NULL). */
wf_status wf_server_poll(wf_server* srv, uint64_t ticket, int32_t* done,
                         wf_solve_info* info);
/* Copies the result (n^3 doubles, host) and releases the ticket.  A failed
 * request returns its error (a cancelled one WF_ESTATE) and writes nothing. */
wf_status wf_server_fetch(wf_server* srv, uint64_t ticket, double* s_out);
/* Stops a queued or running request at its next chunk boundary; poll then
 * reports it done with status WF_ESTATE. */
wf_status wf_server_cancel(wf_server* srv, uint64_t ticket);
wf_status wf_server_stats_get(wf_server* srv, wf_server_stats* stats);
const char* wf_server_last_error(const wf_server* srv);
wf_status wf_server_destroy(wf_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* WIENER_H */
