// HIP kernels of the Wiener-filter hot path for gfx950 (MI355X): CG vector
// updates, mixed-precision reliable updates, gridding and input validation.
// The FFT passes of the operator live in fftpass.hip.
#include "fft.h"
#include "launch.h"
#include "stencil.h"

namespace wf {

// ---------------------------------------------------------------------------
// CG vector kernels (grid-stride with a fixed grid: deterministic partials)
// ---------------------------------------------------------------------------
int vec_blocks(int64_t m) {
  int64_t b = (m + VEC_THREADS * 4 - 1) / (VEC_THREADS * 4);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_cg_init(T* x, T* r, const double* src, int64_t m,
                                                         int64_t rs, double* partials,
                                                         CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  T* xx = x + rhs * rs;
  T* rr = r + rhs * rs;
  const double* ss = src + rhs * rs;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const T v = (T)ss[i];
    rr[i] = v;
    xx[i] = T(0);
    acc += (double)v * (double)v;
  }
  const double part = block_sum(acc, red);
  double* parts = partials + (int64_t)rhs * gridDim.x;
  if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double tot = reduce_partials(parts, gridDim.x, red);
    if (threadIdx.x == 0) {
      st->rho = tot;
      st->rho_old = tot;
      st->bnorm = sqrt(tot);
      st->rel = 1.0;
      st->iter = 0;
      st->first = 1;
      st->pending = 0;
      st->status = CG_RUNNING;
      st->done = (tot == 0.0 || st->max_iter <= 0) ? 1 : 0;
      if (tot == 0.0) st->status = CG_CONVERGED;
      else if (st->max_iter <= 0) st->status = CG_MAXITER;
      reset_ticket(&st->ticket);
    }
  }
}

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// r -= alpha q and the block partial of r.r (x += alpha p waits for the next
// z pass, which reads p anyway).  Each block owns a contiguous run of
// VEC_THREADS * K 16-byte vectors; every load of a thread is issued before
// the first use, and the streams bypass the caches (nontemporal): measured on
// MI355X this moves ~20% more bytes per second than a grid-stride loop.
template <typename T, int K>
__global__ __launch_bounds__(VEC_THREADS) void k_cg_update(T* r, const T* q, int64_t m, int64_t rs,
                                                           double* partials, CgState* st_all) {
  using R = typename Vec16<T>::type;
  constexpr int RW = 16 / sizeof(T);
  __shared__ double red[VEC_THREADS / 64];
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  if (st->done) return;
  const T alpha = (T)st->alpha;
  R* rr = reinterpret_cast<R*>(r + rhs * rs);
  const R* qq = reinterpret_cast<const R*>(q + rhs * rs);
  const int64_t mv = m / RW;
  const int64_t base = (int64_t)blockIdx.x * VEC_THREADS * K + threadIdx.x;
  double acc = 0.0;
  if constexpr (K == 1) {
    if (base < mv) {
      const R rn = __builtin_nontemporal_load(rr + base) - alpha * __builtin_nontemporal_load(qq + base);
      __builtin_nontemporal_store(rn, rr + base);
#pragma unroll
      for (int j = 0; j < RW; ++j) acc += (double)rn[j] * (double)rn[j];
    }
  } else {
    // whole blocks only (the launcher checks that K * VEC_THREADS divides mv)
    (void)mv;
    R rv[K], qv[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int64_t i = base + c * VEC_THREADS;
      rv[c] = __builtin_nontemporal_load(rr + i);
      qv[c] = __builtin_nontemporal_load(qq + i);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int64_t i = base + c * VEC_THREADS;
      const R rn = rv[c] - alpha * qv[c];
      __builtin_nontemporal_store(rn, rr + i);
#pragma unroll
      for (int j = 0; j < RW; ++j) acc += (double)rn[j] * (double)rn[j];
    }
  }
  const double part = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(int64_t)rhs * gridDim.x + blockIdx.x] = part;
}

template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_cg_flush(T* x, const T* p, int64_t m, int64_t rs,
                                                          const CgState* st_all) {
  const int rhs = blockIdx.y;
  const CgState* st = st_all + rhs;
  if (!st->pending) return;
  const T alpha = (T)st->alpha;
  T* xx = x + rhs * rs;
  const T* pp = p + rhs * rs;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride)
    xx[i] = xx[i] + alpha * pp[i];
}

__global__ void k_clear_pending(CgState* st_all) {
  if (threadIdx.x == 0) st_all[blockIdx.x].pending = 0;
}

template <typename T>
hipError_t launch_cg_flush(T* x, const T* p, int64_t m, int64_t rs, CgState* st, int nrhs,
                           hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  klaunch(k_cg_flush<T>, grid, dim3(VEC_THREADS), 0, s, x, p, m, rs, st);
  klaunch(k_clear_pending, dim3(nrhs), dim3(64), 0, s, st);
  return hipGetLastError();
}
template hipError_t launch_cg_flush<float>(float*, const float*, int64_t, int64_t, CgState*, int,
                                           hipStream_t);
template hipError_t launch_cg_flush<double>(double*, const double*, int64_t, int64_t, CgState*, int,
                                            hipStream_t);

__global__ __launch_bounds__(VEC_THREADS) void k_state_norm(const double* v, int64_t m, int64_t rs,
                                                            double* partials, CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  const double* vv = v + rhs * rs;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride)
    acc += vv[i] * vv[i];
  const double part = block_sum(acc, red);
  double* parts = partials + (int64_t)rhs * gridDim.x;
  if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double tot = reduce_partials(parts, gridDim.x, red);
    if (threadIdx.x == 0) {
      st->onorm = sqrt(tot);
      reset_ticket(&st->ticket);
    }
  }
}

hipError_t launch_state_norm(const double* v, int64_t m, int64_t rs, double* partials,
                             CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  klaunch(k_state_norm, grid, dim3(VEC_THREADS), 0, s, v, m, rs, partials, st);
  return hipGetLastError();
}

// vectors per thread of the update kernel: long runs for large grids, one
// vector for small ones (enough blocks to fill 256 CUs)
static int update_k(int64_t m, int rw) {
  const int64_t mv = m / rw, run = (int64_t)VEC_THREADS * 8;
  return (mv >= run * 2048 && mv % run == 0) ? 8 : 1;
}

int update_blocks(int64_t m, bool fp64) {
  const int rw = fp64 ? 2 : 4;
  const int64_t per = (int64_t)VEC_THREADS * update_k(m, rw);
  return (int)((m / rw + per - 1) / per);
}

template <typename T>
hipError_t launch_cg_init(T* x, T* r, const double* src, int64_t m, int64_t rs,
                          double* partials, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  klaunch(k_cg_init<T>, grid, dim3(VEC_THREADS), 0, s, x, r, src, m, rs, partials, st);
  return hipGetLastError();
}
template hipError_t launch_cg_init<float>(float*, float*, const double*, int64_t, int64_t,
                                          double*, CgState*, int, hipStream_t);
template hipError_t launch_cg_init<double>(double*, double*, const double*, int64_t, int64_t,
                                           double*, CgState*, int, hipStream_t);

template <typename T>
hipError_t launch_cg_update(T* r, const T* q, int64_t m, int64_t rs, double* partials,
                            CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(update_blocks(m, sizeof(T) == 8), nrhs);
  if (update_k(m, 16 / sizeof(T)) == 8)
    klaunch((k_cg_update<T, 8>), grid, dim3(VEC_THREADS), 0, s, r, q, m, rs, partials, st);
  else
    klaunch((k_cg_update<T, 1>), grid, dim3(VEC_THREADS), 0, s, r, q, m, rs, partials, st);
  return hipGetLastError();
}
template hipError_t launch_cg_update<float>(float*, const float*, int64_t, int64_t, double*,
                                            CgState*, int, hipStream_t);
template hipError_t launch_cg_update<double>(double*, const double*, int64_t, int64_t, double*,
                                             CgState*, int, hipStream_t);

// ---------------------------------------------------------------------------
// mixed precision: FP32 CG with FP64 reliable updates
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(VEC_THREADS) void k_rel_init(double* x64, double* r64,
                                                          const double* b, float* x32, float* r32,
                                                          int64_t m, int64_t rs, double* partials,
                                                          CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  const int64_t o = rhs * rs;
  double bb = 0.0, rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const double v = b[o + i];
    const float f = (float)v;
    x64[o + i] = 0.0;
    r64[o + i] = v;
    x32[o + i] = 0.f;
    r32[o + i] = f;
    bb += v * v;
    rr += (double)f * (double)f;
  }
  const double pb = block_sum(bb, red);
  const double pr = block_sum(rr, red);
  double* parts = partials + (int64_t)rhs * 2 * gridDim.x;
  if (publish_partial2(pb, pr, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double tb = reduce_partials_strided(parts, gridDim.x, 2, red);
    const double tr = reduce_partials_strided(parts + 1, gridDim.x, 2, red);
    if (threadIdx.x == 0) {
      st->bnorm = sqrt(tb);
      st->outer_rr = tb;
      st->rho = tr;
      st->rho_old = tr;
      st->rmax = sqrt(tr);
      st->rel = tb > 0.0 ? 1.0 : 0.0;
      st->iter = 0;
      st->updates = 0;
      st->first = 1;
      st->pending = 0;
      st->reliable = 1;
      if (tb == 0.0) {
        st->done = 1;
        st->status = CG_CONVERGED;
      } else if (st->max_iter <= 0) {
        st->done = 1;
        st->status = CG_MAXITER;
      } else {
        st->done = 0;
        st->status = CG_RUNNING;
      }
      reset_ticket(&st->ticket);
    }
  }
}

hipError_t launch_rel_init(double* x64, double* r64, const double* b, float* x32, float* r32,
                           int64_t m, int64_t rs, double* partials, CgState* st, int nrhs,
                           hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  klaunch(k_rel_init, grid, dim3(VEC_THREADS), 0, s, x64, r64, b, x32, r32, m, rs,
                     partials, st);
  return hipGetLastError();
}

// Weight of element i (a double of an interleaved half spectrum of the
// prior-split form) in ||C v||^2: the square of the prior-split factor of its
// mode.  Those vectors are stored in the x pass's tile order with tiles of tv
// columns: the main part holds column kz of outer row y at x index x at
// ((y (h / tv) + kz / tv) n + x) tv + kz % tv, the kz = h plane that follows
// it holds column y at ((y / tv) n + x) tv + y % tv (h = n / 2).
__device__ __forceinline__ double split_weight(const double* fac, int n, int tv,
                                              int64_t spec_main, int64_t i) {
  const int64_t ci = i >> 1;
  const int h = n / 2;
  int x, y, kz;
  if (ci < spec_main) {
    const int64_t t = ci / tv;  // (y (h / tv) + kz / tv) n + x
    const int64_t u = t / n;    // y (h / tv) + kz / tv
    const int nb = h / tv;
    x = (int)(t - u * n);
    y = (int)(u / nb);
    kz = (int)(u - (int64_t)y * nb) * tv + (int)(ci - t * tv);
  } else {
    const int64_t cj = ci - spec_main;
    const int64_t t = cj / tv;  // (y / tv) n + x
    const int64_t u = t / n;
    x = (int)(t - u * n);
    y = (int)u * tv + (int)(cj - t * tv);
    kz = h;
  }
  const int mx = x <= h ? x : n - x, my = y <= h ? y : n - y;
  const int kzb = (h + SPLIT_FB) / SPLIT_FB;
  const double c = fac[((int64_t)(my * kzb + kz / SPLIT_FB) * (h + 1) + mx) * SPLIT_FB +
                       kz % SPLIT_FB];
  return c * c;
}

// RHS waiting for an update: x64 += x32 (+ the pending alpha p32), x32 = 0,
// and move = ||fold|| / ||x64 new||, weighted by the prior-split factor
// squared when `fac` is given (then the vectors are half spectra of y and the
// norms are those of s = C y).
__global__ __launch_bounds__(VEC_THREADS) void k_rel_fold(double* x64, float* x32, const float* p32,
                                                          int64_t m, int64_t rs, double* partials,
                                                          const double* fac, int n, int tv,
                                                          int64_t spec_main, int64_t fac_rs,
                                                          CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  if (st->status != CG_UPDATE) return;
  const float alpha = st->pending ? (float)st->alpha : 0.f;
  const int64_t o = rhs * rs;
  const double* fr = fac ? fac + rhs * fac_rs : nullptr;
  double dd = 0.0, xx = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const double d = (double)(x32[o + i] + alpha * p32[o + i]);
    const double xn = x64[o + i] + d;
    x64[o + i] = xn;
    x32[o + i] = 0.f;
    const double wgt = fr ? split_weight(fr, n, tv, spec_main, i) : 1.0;
    dd += wgt * d * d;
    xx += wgt * xn * xn;
  }
  const double pd = block_sum(dd, red);
  const double px = block_sum(xx, red);
  double* parts = partials + (int64_t)rhs * 2 * gridDim.x;
  if (publish_partial2(pd, px, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double td = reduce_partials_strided(parts, gridDim.x, 2, red);
    const double tx = reduce_partials_strided(parts + 1, gridDim.x, 2, red);
    if (threadIdx.x == 0) {
      st->move = tx > 0.0 ? sqrt(td / tx) : 0.0;
      reset_ticket(&st->ticket);
    }
  }
}

hipError_t launch_rel_fold(double* x64, float* x32, const float* p32, int64_t m, int64_t rs,
                           double* partials, const double* fac, int n, int64_t spec_main,
                           int64_t fac_rs, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  const int tv = fac ? split_vec_tile(n) : 1;
  klaunch(k_rel_fold, grid, dim3(VEC_THREADS), 0, s, x64, x32, p32, m, rs, partials,
                     fac, n, tv, spec_main, fac_rs, st);
  return hipGetLastError();
}

// With p32 (the folded FP32 iteration, whose direction for the next step is
// already formed when the update falls due): that direction continues with
// the refreshed residual, p += r_new - r_old; when the update came between
// iterations instead (x += alpha p still pending, folded by the update), the
// next direction restarts from r.
__global__ __launch_bounds__(VEC_THREADS) void k_rel_reset(float* r32, const double* r64,
                                                           float* p32, int64_t m, int64_t rs,
                                                           double* partials, CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  if (st->status != CG_UPDATE) return;
  const bool was_pending = st->pending != 0;
  const bool carry = p32 != nullptr && !was_pending;
  const int64_t o = rhs * rs;
  double rr = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const float f = (float)r64[o + i];
    if (carry) p32[o + i] += f - r32[o + i];
    r32[o + i] = f;
    rr += (double)f * (double)f;
  }
  const double part = block_sum(rr, red);
  double* parts = partials + (int64_t)rhs * gridDim.x;
  if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double tot = reduce_partials(parts, gridDim.x, red);
    if (threadIdx.x == 0) {
      // the folded iteration counts a step when the next iteration applies
      // it; a step the fold applied instead counts here
      if (p32 && was_pending) st->iter += 1;
      st->updates += 1;
      st->upd_iter = st->iter;
      st->pending = 0;  // folded
      const double rel = sqrt(st->outer_rr) / st->bnorm;
      // with err_tol: once the residual meets tol, the solve goes on in
      // windows of the updates that reduce the residual by 10 (hold_need of
      // them) and stops after the first window whose summed changes of the
      // solution are at most err_tol: that change shows the error the
      // residual had hidden
      if (rel <= st->tol) {
        if (st->hold > 0) {
          st->move_acc += st->move;
          st->win += 1;
        }
        st->hold += 1;
      } else {
        st->hold = 0;
        st->win = 0;
        st->move_acc = 0.0;
      }
      const bool window = st->win >= st->hold_need;
      const bool settled = !(st->err_tol > 0.0) || (window && st->move_acc <= st->err_tol);
      if (window && !settled) {  // the next window starts
        st->win = 0;
        st->move_acc = 0.0;
      }
      if (st->updates > 1 && !(rel < 0.9 * st->best_rel)) {
        st->stall += 1;
      } else {
        st->stall = 0;
      }
      if (st->updates == 1 || rel < st->best_rel) st->best_rel = rel;
      if (rel <= st->tol && settled) {
        st->status = CG_CONVERGED;
      } else if (st->iter >= st->max_iter) {
        st->status = CG_MAXITER;
      } else if (st->max_updates > 0 && st->updates >= st->max_updates) {
        st->status = CG_STOPPED;
      } else if (st->stall >= STALL_UPDATES) {
        st->status = CG_STOPPED;
        st->stagnated = 1;
      } else {
        // continue from the refreshed residual with the same direction; with
        // the residual met but the solution still moving, the next update
        // comes when the residual has dropped by delta again
        st->beta = tot / st->rho_old;
        if (p32) st->first = was_pending ? 1 : 0;
        st->rho = tot;
        st->rmax = sqrt(tot);
        st->rel = sqrt(tot) / st->bnorm;
        st->done = 0;
        st->status = CG_RUNNING;
      }
      reset_ticket(&st->ticket);
    }
  }
}

hipError_t launch_rel_reset(float* r32, const double* r64, float* p32, int64_t m, int64_t rs,
                            double* partials, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  klaunch(k_rel_reset, grid, dim3(VEC_THREADS), 0, s, r32, r64, p32, m, rs, partials, st);
  return hipGetLastError();
}

// Initialises the scalar state of a solve whose nbar was written to the device
// by the data-vector kernel (used by the server, which never waits on it).
__global__ void k_state_init(CgState* st_all, const double* nbar, double tol, int32_t max_iter,
                             double delta, int32_t max_updates, double err_tol) {
  if (threadIdx.x != 0) return;
  CgState* st = st_all + blockIdx.x;
  CgState z{};
  z.nbar = nbar[blockIdx.x];
  z.tol = tol;
  z.max_iter = max_iter;
  z.delta = delta;
  z.max_updates = max_updates;
  z.err_tol = err_tol;
  z.hold_need = settle_intervals(delta);
  *st = z;
}

hipError_t launch_state_init(CgState* st, const double* nbar, double tol, int32_t max_iter,
                             double delta, int32_t max_updates, double err_tol, int nrhs,
                             hipStream_t s) {
  klaunch(k_state_init, dim3(nrhs), dim3(64), 0, s, st, nbar, tol, max_iter, delta,
                     max_updates, err_tol);
  return hipGetLastError();
}

// Stops one solve where it stands (a cancelled request): kernels skip it from
// then on.
__global__ void k_state_stop(CgState* st) {
  if (threadIdx.x == 0) {
    st->done = 1;
    st->status = CG_STOPPED;
  }
}

// A running mixed solve asks for a reliable update now (the stepwise API's
// finish between updates).
__global__ void k_state_request_update(CgState* st) {
  if (threadIdx.x == 0 && !st->done) {
    st->done = 1;
    st->status = CG_UPDATE;
  }
}

hipError_t launch_state_request_update(CgState* st, hipStream_t s) {
  klaunch(k_state_request_update, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_state_stop(CgState* st, hipStream_t s) {
  klaunch(k_state_stop, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fills and conversions
// ---------------------------------------------------------------------------
template <typename V> __global__ void k_fill(V* p, int64_t n, V v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
static dim3 fill_grid(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}
hipError_t launch_fill_i64(long long* p, int64_t n, hipStream_t s) {
  klaunch(k_fill<long long>, fill_grid(n), dim3(256), 0, s, p, n, 0LL);
  return hipGetLastError();
}
hipError_t launch_fill_c64(double2* p, int64_t n, hipStream_t s) {
  klaunch(k_fill<double2>, fill_grid(n), dim3(256), 0, s, p, n, double2{0.0, 0.0});
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s) {
  klaunch(k_fill<double>, fill_grid(n), dim3(256), 0, s, p, n, 0.0);
  return hipGetLastError();
}

template <typename O, typename I>
__global__ void k_convert(O* out, const I* in, double unit, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (O)((double)in[i] * unit);
}
hipError_t launch_f64_to_f32(float* out, const double* in, int64_t n, hipStream_t s) {
  klaunch((k_convert<float, double>), fill_grid(n), dim3(256), 0, s, out, in, 1.0, n);
  return hipGetLastError();
}
hipError_t launch_f32_to_f64(double* out, const float* in, int64_t n, hipStream_t s) {
  klaunch((k_convert<double, float>), fill_grid(n), dim3(256), 0, s, out, in, 1.0, n);
  return hipGetLastError();
}
hipError_t launch_i64_to_f64(double* out, const long long* in, double unit, int64_t n,
                             hipStream_t s) {
  klaunch((k_convert<double, long long>), fill_grid(n), dim3(256), 0, s, out, in, unit,
                     n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// galaxies: validation and fixed-point mass assignment (Sec. 3.1.2)
// ---------------------------------------------------------------------------
__global__ void k_check_xyz(const double* xyz, int64_t n3, double box, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    const double v = xyz[i];
    if (!(v >= 0.0 && v < box)) atomicOr(flag, 1);
  }
}

hipError_t launch_check_xyz(const double* xyz, int64_t ngal, double box, int* flag, hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  klaunch(k_check_xyz, fill_grid(3 * ngal), dim3(256), 0, s, xyz, 3 * ngal, box, flag);
  return hipGetLastError();
}

template <int SCHEME>
__global__ __launch_bounds__(256) void k_deposit(const double* __restrict__ xyz, int64_t ngal,
                                                 double c, int nd, unsigned long long* grid) {
  constexpr int S = SCHEME + 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngal) return;
  long long first[3];
  long long w[3][S];
  const double scale = (double)(1LL << FBITS);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double u = __dmul_rn(xyz[3 * g + a], c);
    if (u >= (double)nd) u = u - (double)nd;
    const long long U = (long long)floor(u * scale);
    axis_stencil<SCHEME>(U, first[a], w[a]);
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
    long long ix = (first[0] + i) % nd;
    if (ix < 0) ix += nd;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      long long iy = (first[1] + j) % nd;
      if (iy < 0) iy += nd;
      const long long wxy = w[0][i] * w[1][j];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        long long iz = (first[2] + k) % nd;
        if (iz < 0) iz += nd;
        const unsigned long long wt = (unsigned long long)(wxy * w[2][k]);
        if (wt) atomicAdd(grid + ((ix * nd + iy) * nd + iz), wt);
      }
    }
  }
}

hipError_t launch_deposit(int scheme, const double* xyz, int64_t ngal, double c, int nd,
                          long long* grid, hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  dim3 gridd((unsigned)((ngal + 255) / 256));
  auto* gp = reinterpret_cast<unsigned long long*>(grid);
  switch (scheme) {
    case 0: klaunch(k_deposit<0>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
    case 1: klaunch(k_deposit<1>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
    case 2: klaunch(k_deposit<2>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// mask, prior table, data vector
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(VEC_THREADS) void k_mask(const double* w, double* w64, float* w32,
                                                     int64_t m, int* flag, double* partials,
                                                     uint32_t* ticket, double* sumw) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  double acc = 0.0;
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const double v = w[i];
    if (!(v >= 0.0 && v <= 1.0)) bad = 1;
    w64[i] = v;
    w32[i] = (float)v;
    acc += v;
  }
  if (bad) atomicOr(flag, 1);
  const double part = block_sum(acc, red);
  if (publish_partial(part, partials, ticket, gridDim.x, &last_flag)) {
    const double tot = reduce_partials(partials, gridDim.x, red);
    if (threadIdx.x == 0) {
      *sumw = tot;
      reset_ticket(ticket);
    }
  }
}

hipError_t launch_mask(const double* w, double* w64, float* w32, int64_t m, int* flag,
                       double* partials, uint32_t* ticket, double* sumw, hipStream_t s) {
  klaunch(k_mask, dim3(vec_blocks(m)), dim3(VEC_THREADS), 0, s, w, w64, w32, m, flag,
                     partials, ticket, sumw);
  return hipGetLastError();
}

__global__ void k_lambda(const double* p, int64_t len, double dv, double inv_m, double* lam64,
                         int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len; j += stride) {
    double l = 0.0;
    if (j > 0) {
      const double v = p[j];
      if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
      l = (dv / v) * inv_m;
      if (!isfinite(l)) atomicOr(flag, 1);
    }
    lam64[j] = l;
  }
}

hipError_t launch_lambda(const double* p, int64_t len, double dv, double inv_m, double* lam64,
                         int* flag, hipStream_t s) {
  klaunch(k_lambda, fill_grid(len), dim3(256), 0, s, p, len, dv, inv_m, lam64, flag);
  return hipGetLastError();
}

__global__ void k_data_vector(const double* nobs, const double* w, const double* sumw, double ngal,
                              double* nbar_out, double* b, int64_t m) {
  const double nbar = ngal / *sumw;
  if (blockIdx.x == 0 && threadIdx.x == 0) *nbar_out = nbar;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const double wi = w[i];
    b[i] = wi > 0.0 ? nobs[i] - nbar * wi : 0.0;
  }
}

hipError_t launch_data_vector(const double* nobs, const double* w, const double* sumw, double ngal,
                              double* nbar_out, double* b, int64_t m, hipStream_t s) {
  klaunch(k_data_vector, fill_grid(m), dim3(256), 0, s, nobs, w, sumw, ngal, nbar_out,
                     b, m);
  return hipGetLastError();
}

}  // namespace wf
