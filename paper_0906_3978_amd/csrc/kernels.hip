// HIP kernels of the Wiener-filter hot path for gfx950 (MI355X).
//
// Operator A p = F^-1 Lambda F p + nbar w p (eq:WF with the LSQ noise of
// eq:noiseav) is applied in five sweeps over HBM:
//   1. z pass   : real rows -> half spectrum (two rows per complex FFT),
//                 fused with the CG direction update p = r + beta p;
//   2. y pass   : forward FFT along y (tiles of TB adjacent kz columns);
//   3. x pass   : forward FFT along x, multiply by Lambda[|m|^2], inverse FFT;
//   4. y pass   : inverse FFT along y;
//   5. z pass   : half spectrum -> real rows, fused with + nbar w p and the
//                 partial p.q of the CG step length.
// The half spectrum is stored as main[x][y][kz < N/2] plus the kz = N/2
// plane nyq[x][y], so every strided tile covers an aligned run of columns.
// Reductions are deterministic: each block writes an FP64 partial, the last
// block to finish sums the partials in a fixed order and updates the scalar
// CG state on the device.
#include "fft.h"
#include "launch.h"

namespace wf {

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
template <typename T, int N> constexpr int z_nb() {
  const int elems = (sizeof(T) == 8) ? 2048 : 4096;  // 32 KB of LDS per block
  int lim = elems / N;
  if (lim < 1) lim = 1;
  const int pairs = N * N / 2;
  for (int d = lim; d >= 1; --d)
    if (pairs % d == 0) return d;
  return 1;
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

template <typename T, int N> constexpr int str_tb() {
  const int cap = 65536 / (N * (int)sizeof(cplx<T>));
  int p = 1;
  while (p * 2 <= cap && p < 16) p *= 2;
  return cgcd(p, N / 4);
}

__device__ __forceinline__ int signed_m(int i, int n) { return i < (n >> 1) ? i : i - n; }

// ---------------------------------------------------------------------------
// z forward: real rows -> half spectrum
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_zfwd(ZfwdArgs<T> a) {
  using V = cplx<T>;
  constexpr int NB = z_nb<T, N>();
  constexpr int H = N / 2;
  __shared__ V lds[NB * N];
  const int rhs = blockIdx.y;
  CgState* st = a.st ? a.st + rhs : nullptr;
  if (st && st->done) return;
  const int64_t row0 = (int64_t)blockIdx.x * NB * 2;

  T beta = T(0);
  bool first = true;
  if constexpr (MODE == ZIN_CGP) {
    first = st->first != 0;
    beta = (T)st->beta;
  }
  for (int e = threadIdx.x; e < NB * N; e += NT) {
    const int b = e / N, z = e - b * N;
    const int64_t i0 = (row0 + 2 * b) * N + z, i1 = i0 + N;
    T v0, v1;
    if constexpr (MODE == ZIN_REAL) {
      const T* in = a.in + rhs * a.rhs_in;
      v0 = in[i0];
      v1 = in[i1];
    } else if constexpr (MODE == ZIN_CGP) {
      const T* r = a.in + rhs * a.rhs_in;
      T* p = a.p + rhs * a.rhs_in;
      v0 = first ? r[i0] : r[i0] + beta * p[i0];
      v1 = first ? r[i1] : r[i1] + beta * p[i1];
      p[i0] = v0;
      p[i1] = v1;
    } else {
      const long long* g = a.gin + rhs * a.rhs_in;
      v0 = (T)((double)g[i0] * a.unit);
      v1 = (T)((double)g[i1] * a.unit);
    }
    lds[b * N + z] = V{v0, v1};
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, -1>(lds, a.tw);

  // split the two real rows: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
  V* om = a.out_main + rhs * a.rhs_main;
  V* on = a.out_nyq ? a.out_nyq + rhs * a.rhs_nyq : nullptr;
  const int nk = a.nkz_out;
  for (int e = threadIdx.x; e < NB * (H + 1); e += NT) {
    const int b = e / (H + 1), k = e - b * (H + 1);
    const V zk = lds[b * N + k];
    const V zn = lds[b * N + ((N - k) % N)];
    const V A = {T(0.5) * (zk.x + zn.x), T(0.5) * (zk.y - zn.y)};
    const V B = {T(0.5) * (zk.y + zn.y), T(-0.5) * (zk.x - zn.x)};
    const int64_t r0 = row0 + 2 * b;
    if (k < nk) {
      om[r0 * nk + k] = A;
      om[(r0 + 1) * nk + k] = B;
    } else if (k == H && on) {
      on[r0] = A;
      on[r0 + 1] = B;
    }
  }
}

// ---------------------------------------------------------------------------
// z inverse: half spectrum -> real rows (+ fused CG / residual work)
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_zinv(ZinvArgs<T> a) {
  using V = cplx<T>;
  constexpr int NB = z_nb<T, N>();
  constexpr int H = N / 2;
  __shared__ V lds[NB * N];
  __shared__ double red[NT / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = a.st ? a.st + rhs : nullptr;
  if (MODE == ZOUT_CGQ && st->done) return;
  const int64_t row0 = (int64_t)blockIdx.x * NB * 2;
  const V* im = a.in_main + rhs * a.rhs_main;
  const V* in = a.in_nyq + rhs * a.rhs_nyq;

  for (int e = threadIdx.x; e < NB * N; e += NT) {
    const int b = e / N, k = e - b * N;
    const int kk = k <= H ? k : N - k;
    const int64_t r0 = row0 + 2 * b;
    V A = kk < H ? im[r0 * H + kk] : in[r0];
    V B = kk < H ? im[(r0 + 1) * H + kk] : in[r0 + 1];
    if (k == 0 || k == H) {
      A.y = T(0);
      B.y = T(0);
    } else if (k > H) {
      A.y = -A.y;
      B.y = -B.y;
    }
    lds[b * N + k] = V{A.x - B.y, A.y + B.x};
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, +1>(lds, a.tw);

  double acc = 0.0;
  T* out = a.out + rhs * a.rhs_out;
  T nbar = T(0);
  if constexpr (MODE != ZOUT_REAL) nbar = (T)st->nbar;
  for (int e = threadIdx.x; e < NB * N; e += NT) {
    const int b = e / N, z = e - b * N;
    const V v = lds[b * N + z];
    const int64_t i0 = (row0 + 2 * b) * N + z, i1 = i0 + N;
    if constexpr (MODE == ZOUT_REAL) {
      out[i0] = (T)(v.x * a.scale);
      out[i1] = (T)(v.y * a.scale);
    } else if constexpr (MODE == ZOUT_CGQ || MODE == ZOUT_APPLY) {
      const T* p = a.aux + rhs * a.rhs_aux;
      const T p0 = p[i0], p1 = p[i1];
      const T nw0 = nbar * a.w[i0], nw1 = nbar * a.w[i1];
      const T q0 = v.x + nw0 * p0, q1 = v.y + nw1 * p1;
      out[i0] = q0;
      out[i1] = q1;
      if constexpr (MODE == ZOUT_CGQ) acc += (double)p0 * (double)q0 + (double)p1 * (double)q1;
    } else {  // ZOUT_RES: r = b - A x
      const T* x = a.aux + rhs * a.rhs_aux;
      const double* bb = a.bvec + rhs * a.rhs_b;
      const T nw0 = nbar * a.w[i0], nw1 = nbar * a.w[i1];
      const T r0v = (T)bb[i0] - (v.x + nw0 * x[i0]);
      const T r1v = (T)bb[i1] - (v.y + nw1 * x[i1]);
      out[i0] = r0v;
      out[i1] = r1v;
      acc += (double)r0v * (double)r0v + (double)r1v * (double)r1v;
    }
  }
  if constexpr (MODE == ZOUT_CGQ || MODE == ZOUT_RES) {
    const double part = block_sum(acc, red);
    double* parts = a.partials + (int64_t)rhs * gridDim.x;
    if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
      const double tot = reduce_partials(parts, gridDim.x, red);
      if (threadIdx.x == 0) {
        if constexpr (MODE == ZOUT_CGQ) {
          st->pq = tot;
          if (!(tot > 0.0) || !isfinite(tot)) {
            st->done = 1;
            st->status = CG_BREAKDOWN;
          } else {
            st->alpha = st->rho / tot;
          }
        } else {
          st->outer_rr = tot;
        }
        reset_ticket(&st->ticket);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// strided passes
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_strided(StrArgs<T> a) {
  using V = cplx<T>;
  constexpr int TB = str_tb<T, N>();
  __shared__ V lds[TB * N];
  const int rhs = blockIdx.y;
  if (a.st && a.st[rhs].done) return;
  int blk = blockIdx.x;
  const bool second = blk >= a.nblk0;
  const Seg<T> s = second ? a.s1 : a.s0;
  if (second) blk -= a.nblk0;
  const int outer = blk / s.n_btiles;
  const int b0 = (blk - outer * s.n_btiles) * TB;

  const V* in = s.in + rhs * s.in_rhs + outer * s.in_outer + b0 * s.in_batch;
  if (!s.axis_contig) {
    for (int e = threadIdx.x; e < TB * N; e += NT) {
      const int b = e % TB, i = e / TB;
      lds[e] = in[i * s.in_axis + b * s.in_batch];
    }
  } else {
    for (int e = threadIdx.x; e < TB * N; e += NT) {
      const int i = e % N, b = e / N;
      lds[i * TB + b] = in[i * s.in_axis + b * s.in_batch];
    }
  }
  __syncthreads();
  if constexpr (MODE == SM_INV) fft_tile<T, N, TB, NT, true, +1>(lds, a.tw);
  else fft_tile<T, N, TB, NT, true, -1>(lds, a.tw);

  if constexpr (MODE == SM_FWD_LAM_INV) {
    const int mo = s.lam_outer_signed ? signed_m(outer, N) : 0;
    const int base = mo * mo + s.lam_const;
    for (int e = threadIdx.x; e < TB * N; e += NT) {
      const int b = e % TB, i = e / TB;
      const int mi = signed_m(i, N);
      const int mb = s.lam_batch_signed ? signed_m(b0 + b, N) : (b0 + b);
      const T l = a.lam[base + mi * mi + mb * mb];
      V v = lds[e];
      lds[e] = V{v.x * l, v.y * l};
    }
    __syncthreads();
    fft_tile<T, N, TB, NT, true, +1>(lds, a.tw);
  }

  V* out = s.out + rhs * s.out_rhs + outer * s.out_outer + b0 * s.out_batch;
  if constexpr (MODE == SM_FWD_CROP) {
    const int no = s.n_out, h = no / 2;
    for (int e = threadIdx.x; e < TB * no; e += NT) {
      const int b = e % TB, o = e / TB;
      V v = {T(0), T(0)};
      if (o != h) v = lds[(o < h ? o : o + (N - no)) * TB + b];
      out[o * s.out_axis + b * s.out_batch] = v;
    }
  } else if (!s.axis_contig) {
    for (int e = threadIdx.x; e < TB * N; e += NT) {
      const int b = e % TB, i = e / TB;
      out[i * s.out_axis + b * s.out_batch] = lds[e];
    }
  } else {
    for (int e = threadIdx.x; e < TB * N; e += NT) {
      const int i = e % N, b = e / N;
      out[i * s.out_axis + b * s.out_batch] = lds[i * TB + b];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers (dispatch over the supported lengths)
// ---------------------------------------------------------------------------
#define WF_FOR_LENGTHS(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool fft_length_supported(int n, bool fp64) {
  switch (n) {
#define X(L) case L:
    WF_FOR_LENGTHS(X)
#undef X
    return fp64 || n <= 512;
    default: return false;
  }
}

int strided_tb(int n, bool fp64) {
  switch (n) {
#define X(L) \
  case L: return fp64 ? str_tb<double, L>() : str_tb<float, L>();
    WF_FOR_LENGTHS(X)
#undef X
    default: return 0;
  }
}

int zpass_nb(int n, bool fp64) {
  switch (n) {
#define X(L) \
  case L: return fp64 ? z_nb<double, L>() : z_nb<float, L>();
    WF_FOR_LENGTHS(X)
#undef X
    default: return 0;
  }
}

template <typename T, int N>
static hipError_t zfwd_n(int mode, const ZfwdArgs<T>& a, int64_t nrows, int nrhs, hipStream_t s) {
  constexpr int NB = z_nb<T, N>();
  dim3 grid((unsigned)(nrows / (2 * NB)), (unsigned)nrhs);
  switch (mode) {
    case ZIN_REAL: hipLaunchKernelGGL((k_zfwd<T, N, ZIN_REAL>), grid, dim3(NT), 0, s, a); break;
    case ZIN_CGP: hipLaunchKernelGGL((k_zfwd<T, N, ZIN_CGP>), grid, dim3(NT), 0, s, a); break;
    case ZIN_I64:
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_zfwd<T, N, ZIN_I64>), grid, dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t zinv_n(int mode, const ZinvArgs<T>& a, int64_t nrows, int nrhs, hipStream_t s) {
  constexpr int NB = z_nb<T, N>();
  dim3 grid((unsigned)(nrows / (2 * NB)), (unsigned)nrhs);
  switch (mode) {
    case ZOUT_REAL: hipLaunchKernelGGL((k_zinv<T, N, ZOUT_REAL>), grid, dim3(NT), 0, s, a); break;
    case ZOUT_CGQ: hipLaunchKernelGGL((k_zinv<T, N, ZOUT_CGQ>), grid, dim3(NT), 0, s, a); break;
    case ZOUT_RES: hipLaunchKernelGGL((k_zinv<T, N, ZOUT_RES>), grid, dim3(NT), 0, s, a); break;
    case ZOUT_APPLY: hipLaunchKernelGGL((k_zinv<T, N, ZOUT_APPLY>), grid, dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t strided_n(int mode, const StrArgs<T>& a, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)(a.nblk0 + a.nblk1), (unsigned)nrhs);
  switch (mode) {
    case SM_FWD: hipLaunchKernelGGL((k_strided<T, N, SM_FWD>), grid, dim3(NT), 0, s, a); break;
    case SM_INV: hipLaunchKernelGGL((k_strided<T, N, SM_INV>), grid, dim3(NT), 0, s, a); break;
    case SM_FWD_LAM_INV:
      hipLaunchKernelGGL((k_strided<T, N, SM_FWD_LAM_INV>), grid, dim3(NT), 0, s, a);
      break;
    case SM_FWD_CROP: hipLaunchKernelGGL((k_strided<T, N, SM_FWD_CROP>), grid, dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP32 kernels are only instantiated for target grids (<= 512).
#define WF_FOR_F32(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

template <> hipError_t launch_zfwd<double>(int n, int mode, const ZfwdArgs<double>& a, int64_t nrows,
                                           int nrhs, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return zfwd_n<double, L>(mode, a, nrows, nrhs, s);
    WF_FOR_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template <> hipError_t launch_zfwd<float>(int n, int mode, const ZfwdArgs<float>& a, int64_t nrows,
                                          int nrhs, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return zfwd_n<float, L>(mode, a, nrows, nrhs, s);
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template <> hipError_t launch_zinv<double>(int n, int mode, const ZinvArgs<double>& a, int64_t nrows,
                                           int nrhs, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return zinv_n<double, L>(mode, a, nrows, nrhs, s);
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template <> hipError_t launch_zinv<float>(int n, int mode, const ZinvArgs<float>& a, int64_t nrows,
                                          int nrhs, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return zinv_n<float, L>(mode, a, nrows, nrhs, s);
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template <> hipError_t launch_strided<double>(int n, int mode, const StrArgs<double>& a, int nrhs,
                                              hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return strided_n<double, L>(mode, a, nrhs, s);
    WF_FOR_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template <> hipError_t launch_strided<float>(int n, int mode, const StrArgs<float>& a, int nrhs,
                                             hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return strided_n<float, L>(mode, a, nrhs, s);
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

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
                                                         int64_t rs, int scaled, double* partials,
                                                         CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  const double sc = scaled ? st->scale : 1.0;
  T* xx = x + rhs * rs;
  T* rr = r + rhs * rs;
  const double* ss = src + rhs * rs;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const T v = (T)(ss[i] * sc);
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
      st->bnorm = sqrt(tot);
      st->rel = 1.0;
      st->iter = 0;
      st->first = 1;
      st->status = CG_RUNNING;
      st->done = (tot == 0.0 || st->max_iter <= 0) ? 1 : 0;
      if (tot == 0.0) st->status = CG_CONVERGED;
      else if (st->max_iter <= 0) st->status = CG_MAXITER;
      reset_ticket(&st->ticket);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_cg_update(T* x, T* r, const T* p, const T* q,
                                                           int64_t m, int64_t rs, double* partials,
                                                           CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  if (st->done) return;
  const T alpha = (T)st->alpha;
  T* xx = x + rhs * rs;
  T* rr = r + rhs * rs;
  const T* pp = p + rhs * rs;
  const T* qq = q + rhs * rs;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    xx[i] = xx[i] + alpha * pp[i];
    const T rv = rr[i] - alpha * qq[i];
    rr[i] = rv;
    acc += (double)rv * (double)rv;
  }
  const double part = block_sum(acc, red);
  double* parts = partials + (int64_t)rhs * gridDim.x;
  if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double rho_new = reduce_partials(parts, gridDim.x, red);
    if (threadIdx.x == 0) {
      st->iter += 1;
      st->total_iter += 1;
      const double rel = sqrt(rho_new) / st->bnorm;
      st->rel = rel;
      if (rel <= st->tol) {
        st->done = 1;
        st->status = CG_CONVERGED;
      } else if (st->iter >= st->max_iter) {
        st->done = 1;
        st->status = CG_MAXITER;
      }
      st->beta = rho_new / st->rho;
      st->rho = rho_new;
      st->first = 0;
      reset_ticket(&st->ticket);
    }
  }
}

template <typename T>
hipError_t launch_cg_init(T* x, T* r, const double* src, int64_t m, int64_t rs, int scaled,
                          double* partials, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  hipLaunchKernelGGL(k_cg_init<T>, grid, dim3(VEC_THREADS), 0, s, x, r, src, m, rs, scaled,
                     partials, st);
  return hipGetLastError();
}
template hipError_t launch_cg_init<float>(float*, float*, const double*, int64_t, int64_t, int,
                                          double*, CgState*, int, hipStream_t);
template hipError_t launch_cg_init<double>(double*, double*, const double*, int64_t, int64_t, int,
                                           double*, CgState*, int, hipStream_t);

template <typename T>
hipError_t launch_cg_update(T* x, T* r, const T* p, const T* q, int64_t m, int64_t rs,
                            double* partials, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  hipLaunchKernelGGL(k_cg_update<T>, grid, dim3(VEC_THREADS), 0, s, x, r, p, q, m, rs, partials, st);
  return hipGetLastError();
}
template hipError_t launch_cg_update<float>(float*, float*, const float*, const float*, int64_t,
                                            int64_t, double*, CgState*, int, hipStream_t);
template hipError_t launch_cg_update<double>(double*, double*, const double*, const double*,
                                             int64_t, int64_t, double*, CgState*, int, hipStream_t);

__global__ __launch_bounds__(VEC_THREADS) void k_refine_add(double* x, const float* e, int64_t m,
                                                            int64_t rs, const CgState* st_all) {
  const int rhs = blockIdx.y;
  const CgState* st = st_all + rhs;
  const double sc = sqrt(st->outer_rr);
  double* xx = x + rhs * rs;
  const float* ee = e + rhs * rs;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride)
    xx[i] += sc * (double)ee[i];
}

hipError_t launch_refine_add(double* x, const float* e, int64_t m, int64_t rs, const CgState* st,
                             int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  hipLaunchKernelGGL(k_refine_add, grid, dim3(VEC_THREADS), 0, s, x, e, m, rs, st);
  return hipGetLastError();
}

__global__ __launch_bounds__(VEC_THREADS) void k_outer_init(double* x, double* r, const double* b,
                                                            int64_t m, int64_t rs, double* partials,
                                                            CgState* st_all) {
  __shared__ double red[VEC_THREADS / 64];
  __shared__ int last_flag;
  const int rhs = blockIdx.y;
  CgState* st = st_all + rhs;
  double* xx = x + rhs * rs;
  double* rr = r + rhs * rs;
  const double* bb = b + rhs * rs;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * VEC_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * VEC_THREADS + threadIdx.x; i < m; i += stride) {
    const double v = bb[i];
    rr[i] = v;
    xx[i] = 0.0;
    acc += v * v;
  }
  const double part = block_sum(acc, red);
  double* parts = partials + (int64_t)rhs * gridDim.x;
  if (publish_partial(part, parts, &st->ticket, gridDim.x, &last_flag)) {
    const double tot = reduce_partials(parts, gridDim.x, red);
    if (threadIdx.x == 0) {
      st->outer_rr = tot;
      st->outer_bnorm = sqrt(tot);
      reset_ticket(&st->ticket);
    }
  }
}

hipError_t launch_outer_init(double* x, double* r, const double* b, int64_t m, int64_t rs,
                             double* partials, CgState* st, int nrhs, hipStream_t s) {
  dim3 grid(vec_blocks(m), nrhs);
  hipLaunchKernelGGL(k_outer_init, grid, dim3(VEC_THREADS), 0, s, x, r, b, m, rs, partials, st);
  return hipGetLastError();
}

// Starts the next inner solve of every RHS whose refinement is still running:
// checks the outer residual against outer_tol and the iteration budget,
// then sets the inner tolerance and scale 1/||r_outer||.
__global__ void k_inner_setup(CgState* st_all, double tol) {
  CgState* st = st_all + blockIdx.x;
  if (threadIdx.x != 0) return;
  const double rel = st->outer_bnorm > 0.0 ? sqrt(st->outer_rr) / st->outer_bnorm : 0.0;
  if (st->outer_status == CG_RUNNING) {
    if (rel <= st->outer_tol) st->outer_status = CG_CONVERGED;
    else if (st->budget <= 0) st->outer_status = CG_MAXITER;
  }
  const bool active = st->outer_status == CG_RUNNING;
  st->scale = (active && st->outer_rr > 0.0) ? 1.0 / sqrt(st->outer_rr) : 0.0;
  st->tol = tol;
  st->max_iter = active ? st->budget : 0;
  st->iter = 0;
  st->done = 0;
  st->status = CG_RUNNING;
  st->first = 1;
}

hipError_t launch_inner_setup(CgState* st, double tol, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_setup, dim3(nrhs), dim3(64), 0, s, st, tol);
  return hipGetLastError();
}

__global__ void k_inner_finish(CgState* st_all) {
  CgState* st = st_all + blockIdx.x;
  if (threadIdx.x != 0 || st->outer_status != CG_RUNNING) return;
  st->budget -= st->iter;
  st->outer_steps += 1;
  if (st->status == CG_BREAKDOWN) st->outer_status = CG_BREAKDOWN;
}

hipError_t launch_inner_finish(CgState* st, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_finish, dim3(nrhs), dim3(64), 0, s, st);
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
  hipLaunchKernelGGL(k_fill<long long>, fill_grid(n), dim3(256), 0, s, p, n, 0LL);
  return hipGetLastError();
}
hipError_t launch_fill_c64(double2* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double2>, fill_grid(n), dim3(256), 0, s, p, n, double2{0.0, 0.0});
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, fill_grid(n), dim3(256), 0, s, p, n, 0.0);
  return hipGetLastError();
}

template <typename O, typename I>
__global__ void k_convert(O* out, const I* in, double unit, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (O)((double)in[i] * unit);
}
hipError_t launch_f64_to_f32(float* out, const double* in, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<float, double>), fill_grid(n), dim3(256), 0, s, out, in, 1.0, n);
  return hipGetLastError();
}
hipError_t launch_f32_to_f64(double* out, const float* in, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), fill_grid(n), dim3(256), 0, s, out, in, 1.0, n);
  return hipGetLastError();
}
hipError_t launch_i64_to_f64(double* out, const long long* in, double unit, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, long long>), fill_grid(n), dim3(256), 0, s, out, in, unit,
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
  hipLaunchKernelGGL(k_check_xyz, fill_grid(3 * ngal), dim3(256), 0, s, xyz, 3 * ngal, box, flag);
  return hipGetLastError();
}

constexpr int FBITS = 24;
constexpr int QBITS = 13;

// Per-axis stencil: first node and integer weights (units 2^-13; NGP: 1).
template <int SCHEME>
__device__ __forceinline__ void axis_stencil(long long U, long long& first, long long* w) {
  constexpr long long half = 1LL << (FBITS - 1);
  constexpr long long one = 1LL << QBITS;
  if constexpr (SCHEME == 0) {
    first = (U + half) >> FBITS;
    w[0] = 1;
  } else if constexpr (SCHEME == 1) {
    first = U >> FBITS;
    const long long f = U & ((1LL << FBITS) - 1);
    const long long w1 = (f + (1LL << (FBITS - QBITS - 1))) >> (FBITS - QBITS);
    w[0] = one - w1;
    w[1] = w1;
  } else {
    const long long node = (U + half) >> FBITS;
    const long long d = U - (node << FBITS);
    constexpr int sh = 2 * FBITS + 1 - QBITS;
    constexpr long long rnd = 1LL << (sh - 1);
    const long long a = half - d, b = half + d;
    const long long wm = (a * a + rnd) >> sh;
    const long long wp = (b * b + rnd) >> sh;
    first = node - 1;
    w[0] = wm;
    w[1] = one - wm - wp;
    w[2] = wp;
  }
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
    case 0: hipLaunchKernelGGL(k_deposit<0>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
    case 1: hipLaunchKernelGGL(k_deposit<1>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
    case 2: hipLaunchKernelGGL(k_deposit<2>, gridd, dim3(256), 0, s, xyz, ngal, c, nd, gp); break;
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
  hipLaunchKernelGGL(k_mask, dim3(vec_blocks(m)), dim3(VEC_THREADS), 0, s, w, w64, w32, m, flag,
                     partials, ticket, sumw);
  return hipGetLastError();
}

__global__ void k_lambda(const double* p, int64_t len, double dv, double inv_m, double* lam64,
                         float* lam32, int* flag) {
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
    lam32[j] = (float)l;
  }
}

hipError_t launch_lambda(const double* p, int64_t len, double dv, double inv_m, double* lam64,
                         float* lam32, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, fill_grid(len), dim3(256), 0, s, p, len, dv, inv_m, lam64, lam32,
                     flag);
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
  hipLaunchKernelGGL(k_data_vector, fill_grid(m), dim3(256), 0, s, nobs, w, sumw, ngal, nbar_out,
                     b, m);
  return hipGetLastError();
}

}  // namespace wf
