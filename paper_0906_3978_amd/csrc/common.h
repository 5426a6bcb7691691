// Shared device helpers: complex arithmetic, deterministic block reductions,
// the per-solve scalar state that lives on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wf {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };
template <typename T> using cplx = typename C2<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return {a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return {a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (dir = -1) or +i (dir = +1)
template <int DIR, typename V> __device__ __forceinline__ V mul_i(V a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// ---------------------------------------------------------------------------
// Scalar state of one CG solve (one right-hand side), resident on the device.
// Kernels read the scalars they need and skip all work once `done` is set, so
// the host may enqueue iterations ahead of its convergence checks.
// ---------------------------------------------------------------------------
struct CgState {
  double rho;        // r.r of the current (recursive) residual
  double rho_old;    // r.r of the previous iteration
  double bnorm;      // ||b||
  double tol;        // stop when ||r|| / ||b|| <= tol
  double alpha, beta, pq;
  double rel;        // last ||r|| / ||b|| (recursive)
  double nbar;       // mean density per cell of this right-hand side
  double outer_rr;   // ||b - A64 x64||^2 from the last FP64 residual
  double rmax;       // reliable updates: ||r|| right after the last update
  double delta;      // reliable updates: update once ||r|| <= delta * rmax
  int32_t iter;      // completed CG iterations
  int32_t max_iter;
  int32_t done;      // 1: iteration stopped (converged, max_iter, breakdown, update due)
  int32_t status;    // CG_* below
  int32_t first;     // 1: next direction update is p = r
  int32_t reliable;  // 1: FP32 CG with FP64 reliable updates
  uint32_t ticket;   // last-block counter of the reductions
  int32_t updates;   // reliable updates done
  int32_t max_updates;
  int32_t pending;   // 1: x still lacks alpha p of the last iteration (applied by the next
                     // z pass, a reliable-update fold or a flush)
  double onorm;      // prior-split solves: ||b|| of the original system (bnorm is ||C b||)
  // reliable updates: relative change of the solution s made by the last fold,
  // ||s_new - s_old|| / ||s_new|| (prior-split: measured on s = C y), and the
  // bound it must meet, besides the residual tolerance, to stop (0: none)
  double move;
  double err_tol;
  int32_t hold;      // updates so far, this one included, whose residual met tol
  int32_t hold_need; // intervals the change is summed over: a residual drop of 10 at delta
  double move_acc;   // sum of the changes of the updates in the current window
  double best_rel;   // smallest FP64 relative residual of the reliable updates so far
  int32_t stall;     // consecutive updates that did not improve on best_rel by 10 %
  int32_t stagnated; // 1: stopped because the FP64 residual no longer falls
  int32_t upd_iter;  // iteration count at the last reliable update
  int32_t win;       // updates summed into move_acc in the current window
  double pp;         // folded FP32 iteration: p.p of the direction without its monopole
};

// Reliable updates in a row that do not bring the FP64 residual 10 % below
// its best so far (while the FP32 one fell by 1/delta each time) after which
// a mixed solve stops as stagnated: its tolerance is below what the
// arithmetic can reach.
constexpr int32_t STALL_UPDATES = 4;

// Reliable-update intervals that together reduce the recursive residual by
// at least 10 (each reduces it by delta).
__host__ __device__ inline int32_t settle_intervals(double delta) {
  if (!(delta > 0.0) || delta >= 1.0) return 1;
  const int32_t k = (int32_t)ceil(log(0.1) / log(delta) - 1e-9);
  return k < 1 ? 1 : k;
}

// The prior-split factor table is stored in blocks of this many consecutive kz.
constexpr int SPLIT_FB = 16;

enum : int32_t {
  CG_RUNNING = 0, CG_CONVERGED = 1, CG_MAXITER = 2, CG_BREAKDOWN = 3, CG_STOPPED = 4,
  CG_UPDATE = 5   // reliable update due: fold x into FP64, recompute the residual
};

// Which right-hand sides a launch skips: none, those whose iteration has
// stopped, or all but those waiting for a reliable update.
enum : int32_t { SKIP_NONE = 0, SKIP_DONE = 1, SKIP_UNLESS_UPDATE = 2 };

__device__ __forceinline__ bool skip_rhs(const CgState* st, int mode) {
  if (mode == SKIP_DONE) return st->done != 0;
  if (mode == SKIP_UNLESS_UPDATE) return st->status != CG_UPDATE;
  return false;
}

// Coherent (device-scope) load of a value written by another workgroup of
// the same kernel before its release fence.
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over a 64-lane wavefront (fixed butterfly order: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum, fixed order; every thread gets the result.  `sh` holds
// blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// Writes this block's partial sum; returns true in the block that arrives
// last (all partials visible to it).  The caller then calls
// reduce_partials() and finishes the scalar update.  `flag` is LDS.
__device__ __forceinline__ bool publish_partial(double part, double* partials,
                                                uint32_t* ticket, uint32_t nblocks,
                                                int* flag) {
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = part;
    __threadfence();
    uint32_t t = atomicAdd(ticket, 1u);
    *flag = (t == nblocks - 1);
  }
  __syncthreads();
  bool last = *flag != 0;
  if (last) __threadfence();
  return last;
}

// Two partial sums per block (stored interleaved).
__device__ __forceinline__ bool publish_partial2(double a, double b, double* partials,
                                                 uint32_t* ticket, uint32_t nblocks, int* flag) {
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
    __threadfence();
    uint32_t t = atomicAdd(ticket, 1u);
    *flag = (t == nblocks - 1);
  }
  __syncthreads();
  bool last = *flag != 0;
  if (last) __threadfence();
  return last;
}

// Deterministic sum of partials[0..n): each thread sums a fixed strided
// subset, then a fixed tree.
__device__ __forceinline__ double reduce_partials(const double* partials, uint32_t n,
                                                  double* sh) {
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s += load_agent(partials + i);
  return block_sum(s, sh);
}

__device__ __forceinline__ double reduce_partials_strided(const double* partials, uint32_t n,
                                                          int stride, double* sh) {
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s += load_agent(partials + (size_t)i * stride);
  return block_sum(s, sh);
}

__device__ __forceinline__ void reset_ticket(uint32_t* ticket) {
  __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace wf
