// Solve drivers: FP64 conjugate gradients, mixed-precision iterative
// refinement, the multi-RHS batch, checkpoint/resume.
#pragma once

#include "internal.h"

namespace wf {

Status validate_opts(const wf_solve_opts& o);
// The solution-change bound of a mixed solve (wf_solve_opts.err_tol: 0 gives
// this default, a negative value none); 0 (none) for FP64 solves.
constexpr double DEFAULT_ERR_TOL = 5e-7;
double effective_err_tol(const wf_solve_opts& o);

struct SolveRequest {
  const OperatorData* od = nullptr;
  const Allocator* al = nullptr;
  SolveWork* work = nullptr;   // b64 holds nrhs right-hand sides
  int nrhs = 1;
  const double* nbar = nullptr;  // nrhs values
  wf_solve_opts opts{};
  hipStream_t stream = nullptr;
};

// Solves every RHS from x = 0; x64 of the work holds the solutions.
// Returns the worst status; infos[i] per RHS.
Status run_solve(const SolveRequest& rq, wf_solve_info* infos);

// Asynchronous building blocks (no host synchronisation): the CG states
// must already hold tol, max_iter, delta, max_updates and nbar.
Status solve_start(const OperatorData& od, SolveWork& sw, int nr, bool mixed, hipStream_t s);
Status solve_chunk(const OperatorData& od, SolveWork& sw, int nr, bool mixed, int iters,
                   hipStream_t s);
// mixed: reliable update of the RHS whose state asks for one
Status solve_update(const OperatorData& od, SolveWork& sw, int nr, hipStream_t s);
// after the iterations: FP64 plain CG applies the pending step and puts
// ||b - A x||^2 into outer_rr; prior-split solves (either precision) also
// turn the half-spectrum y into s = C y in x64; plain mixed solves need nothing
Status solve_finish(const OperatorData& od, SolveWork& sw, int nr, bool mixed, hipStream_t s);
void solve_infos(const CgState* st, int nr, bool mixed, bool split, const Grid& g, double ms,
                 wf_solve_info* infos);

// Stepwise solve of one RHS (checkpoint / resume), FP64 or mixed, plain or
// prior-split.  step_iterations runs `iters` more CG iterations (mixed: FP32
// iterations, with the reliable updates the state asks for); step_finish
// (mixed: after folding a pending FP32 correction) writes s into x64.
Status step_begin(const OperatorData& od, const Allocator& al, SolveWork& sw, double nbar,
                  const wf_solve_opts& o, hipStream_t s);
Status step_iterations(const OperatorData& od, SolveWork& sw, int iters, bool mixed,
                       hipStream_t s);
Status step_finish(const OperatorData& od, SolveWork& sw, bool mixed, hipStream_t s,
                   wf_solve_info* info);
size_t snapshot_bytes(const Grid& g, bool split, bool mixed);
// the form of a snapshot from its header (at least its header's bytes); false
// if it is not a snapshot
bool snapshot_kind(const void* buf, bool* split, bool* mixed);
Status snapshot_save(const Grid& g, SolveWork& sw, bool mixed, void* buf, hipStream_t s);
Status snapshot_load(const OperatorData& od, const Allocator& al, SolveWork& sw, const void* buf,
                     hipStream_t s);

struct BatchInputs {
  int nrhs = 0;
  const double* const* xyz = nullptr;
  const int64_t* n_gal = nullptr;
  int scheme = 0;
  int ss = 1;
  wf_mem mem = WF_HOST;
};
Status run_batch(const OperatorData& od, const Allocator& al, DepositWork& dw,
                 const BatchInputs& bi, const wf_solve_opts& o, double* const* s_out,
                 wf_solve_info* infos, double sumw, hipStream_t s);

size_t footprint_bytes(int n, int ss, wf_precision prec, int nrhs, bool split);

int severity(wf_status s);

// signal-dependent noise solves (sd.hip)
constexpr int SD_CHUNK = 16;   // RHS per batched solve
struct SdRequest {
  OperatorData* od = nullptr;
  const Allocator* al = nullptr;
  const double* xyz = nullptr;  // device, n_gal x 3
  int64_t n_gal = 0;
  const double* nobs = nullptr;  // device, n^3
  double nbar = 0.0;
  int kind = WF_NOISE_SD_MEAN;
  double alpha = 0.0;
  uint64_t seed = 0;
  int64_t first = 0;
  int nsamples = 1;
  wf_solve_opts opts{};
  double* mean_out = nullptr;
  double* samples_out = nullptr;
  wf_mem mem = WF_HOST;
  int* flag = nullptr;  // device int
  hipStream_t stream = nullptr;
};
Status run_sd(const SdRequest& rq, wf_solve_info* infos);
hipError_t launch_sd_counts(bool thin, const double* xyz, int64_t ngal, double ct, int n,
                            const double* w, double alpha, uint64_t seed, int64_t first, int K,
                            int32_t* counts, int* flag, hipStream_t s);

}  // namespace wf
