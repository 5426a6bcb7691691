// The five sweeps of the Wiener operator A p = F^-1 Lambda F p + nbar w p
// (eq:WF with the LSQ noise of eq:noiseav) on gfx950:
//   1. z pass : real rows -> half spectrum (two real rows per complex FFT),
//               fused with the CG direction update p = r + beta p;
//   2. y pass : forward FFT along y (tiles of TB adjacent kz columns);
//   3. x pass : forward FFT along x, multiply by Lambda[|m|^2], inverse FFT;
//   4. y pass : inverse FFT along y;
//   5. z pass : half spectrum -> real rows, fused with + nbar w p and the
//               block partial of p.q.
// The half spectrum is stored as main[x][y][kz < N/2] plus the kz = N/2
// plane nyq[x][y], so every strided tile covers an aligned run of columns.
// Global memory is moved in 16-byte vectors, all loads of a thread issued
// before their first use.  Block partials of the reductions are summed in a
// fixed order by a one-block finalize kernel per right-hand side.
#include <algorithm>

#include "fft.h"
#include "launch.h"

namespace wf {

constexpr int NT = 256;

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T> using vec16 = typename Vec16<T>::type;

// 16-byte global accesses; every array a pass touches is streamed once, so
// they bypass the caches (nontemporal).
template <typename T> __device__ __forceinline__ vec16<T> ld16(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const vec16<T>*>(p));
}
template <typename T> __device__ __forceinline__ void st16(T* p, vec16<T> v) {
  __builtin_nontemporal_store(v, reinterpret_cast<vec16<T>*>(p));
}
// Cached 16-byte accesses (the y passes run faster with them).
template <bool NTA, typename T> __device__ __forceinline__ vec16<T> ld16x(const T* p) {
  if constexpr (NTA) return ld16(p);
  else return *reinterpret_cast<const vec16<T>*>(p);
}
template <bool NTA, typename T> __device__ __forceinline__ void st16x(T* p, vec16<T> v) {
  if constexpr (NTA) st16(p, v);
  else *reinterpret_cast<vec16<T>*>(p) = v;
}

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
template <typename T, int N> constexpr int z_nb() {
  const int elems = (sizeof(T) == 8) ? 2048 : 4096;  // 32 KB of LDS per block
  int lim = elems / N;
  if (lim < 1) lim = 1;
  const int pairs = N * N / 2;
  // small grids: fewer pencils per block, so that a pass still spreads over
  // at least 512 blocks (two per CU) where the grid has that many pairs; a
  // 32^3 grid otherwise ran its z passes on 8 blocks
  if (pairs / 512 < lim) lim = pairs / 512 > 1 ? pairs / 512 : 1;
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
  using R = vec16<T>;
  constexpr int RW = 16 / sizeof(T);   // reals per vector
  constexpr int CW = 16 / sizeof(V);   // complex values per vector
  constexpr int NB = z_nb<T, N>();
  constexpr int H = N / 2;
  constexpr int ITEMS = NB * N / RW;
  constexpr int PER = (ITEMS + NT - 1) / NT;
  __shared__ __align__(16) V lds[NB * N];
  __shared__ V twl[N];
  const int rhs = blockIdx.y;
  CgState* st = a.st ? a.st + rhs : nullptr;
  if (st && skip_rhs(st, a.skip)) return;
  const int64_t row0 = (int64_t)blockIdx.x * NB * 2;
  load_twiddles<T, N, NT>(twl, a.tw);

  T beta = T(0), alpha = T(0);
  bool first = true, pending = false;
  if constexpr (MODE == ZIN_CGP) {
    first = st->first != 0;
    beta = (T)st->beta;
    alpha = (T)st->alpha;
    pending = st->pending != 0;
  }
  R va[PER], vb[PER];
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (N / RW), z = (q - b * (N / RW)) * RW;
      const int64_t i0 = (row0 + 2 * b) * N + z;
      if constexpr (MODE == ZIN_REAL) {
        const T* in = a.in + rhs * a.rhs_in;
        va[c] = ld16(in + i0);
        vb[c] = ld16(in + i0 + N);
      } else if constexpr (MODE == ZIN_CGP) {
        const T* r = a.in + rhs * a.rhs_in;
        T* p = a.p + rhs * a.rhs_in;
        va[c] = ld16(r + i0);
        vb[c] = ld16(r + i0 + N);
        if (!first) {
          const R p0 = ld16(p + i0), p1 = ld16(p + i0 + N);
          if (pending) {  // x += alpha p of the previous iteration
            T* x = a.x + rhs * a.rhs_in;
            st16(x + i0, ld16(x + i0) + alpha * p0);
            st16(x + i0 + N, ld16(x + i0 + N) + alpha * p1);
          }
          va[c] += beta * p0;
          vb[c] += beta * p1;
        }
        st16(p + i0, va[c]);
        st16(p + i0 + N, vb[c]);
      } else {
        if constexpr (sizeof(T) == 8) {
          const long long* g = a.gin + rhs * a.rhs_in;
          const double u = a.unit;
          va[c] = R{(double)g[i0] * u, (double)g[i0 + 1] * u};
          vb[c] = R{(double)g[i0 + N] * u, (double)g[i0 + N + 1] * u};
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (N / RW), z = (q - b * (N / RW)) * RW;
#pragma unroll
      for (int j = 0; j < RW; ++j) lds[b * N + z + j] = V{va[c][j], vb[c][j]};
    }
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, -1>(lds, twl);

  // split the two real rows: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
  V* om = a.out_main + rhs * a.rhs_main;
  const int nk = a.nkz_out;
  constexpr int ITEMS2 = NB * H / CW;
  constexpr int PER2 = (ITEMS2 + NT - 1) / NT;
#pragma unroll
  for (int c = 0; c < PER2; ++c) {
    const int q = threadIdx.x + c * NT;
    if (!(ITEMS2 % NT == 0 || q < ITEMS2)) continue;
    const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
    if (k0 >= nk) continue;
    R oa, ob;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int k = k0 + j;
      const V zk = lds[b * N + k];
      const V zn = lds[b * N + ((N - k) % N)];
      oa[2 * j] = T(0.5) * (zk.x + zn.x);
      oa[2 * j + 1] = T(0.5) * (zk.y - zn.y);
      ob[2 * j] = T(0.5) * (zk.y + zn.y);
      ob[2 * j + 1] = T(-0.5) * (zk.x - zn.x);
    }
    const int64_t r0 = row0 + 2 * b;
    st16(reinterpret_cast<T*>(om + r0 * nk + k0), oa);
    st16(reinterpret_cast<T*>(om + (r0 + 1) * nk + k0), ob);
  }
  if (a.out_nyq) {
    V* on = a.out_nyq + rhs * a.rhs_nyq;
    for (int b = threadIdx.x; b < NB; b += NT) {
      const V zh = lds[b * N + H];
      const int64_t r0 = row0 + 2 * b;
      on[r0] = V{zh.x, T(0)};
      on[r0 + 1] = V{zh.y, T(0)};
    }
  }
}

// ---------------------------------------------------------------------------
// z inverse: half spectrum -> real rows (+ fused CG / residual work)
// ---------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ __launch_bounds__(NT) void k_zinv(ZinvArgs<T> a) {
  using V = cplx<T>;
  using R = vec16<T>;
  constexpr int RW = 16 / sizeof(T);
  constexpr int CW = 16 / sizeof(V);
  constexpr int NB = z_nb<T, N>();
  constexpr int H = N / 2;
  __shared__ __align__(16) V lds[NB * N];
  __shared__ V twl[N];
  __shared__ double red[NT / 64];
  const int rhs = blockIdx.y;
  CgState* st = a.st ? a.st + rhs : nullptr;
  if (st && skip_rhs(st, a.skip)) return;
  const int64_t row0 = (int64_t)blockIdx.x * NB * 2;
  load_twiddles<T, N, NT>(twl, a.tw);
  const V* im = a.in_main + rhs * a.rhs_main;
  const V* inq = a.in_nyq + rhs * a.rhs_nyq;

  // Z_k = A_k + i B_k for k <= N/2 and Z_{N-k} = conj A_k + i conj B_k: every
  // spectrum value is read once and written to both places.  Only the real
  // parts of the k = 0 and k = N/2 entries enter (as in a real inverse DFT).
  constexpr int ITEMS = NB * H / CW;
  constexpr int PER = (ITEMS + NT - 1) / NT;
  R va[PER], vb[PER];
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
      const int64_t r0 = row0 + 2 * b;
      va[c] = ld16(reinterpret_cast<const T*>(im + r0 * H + k0));
      vb[c] = ld16(reinterpret_cast<const T*>(im + (r0 + 1) * H + k0));
    }
  }
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        const int k = k0 + j;
        const T ax = va[c][2 * j], ay = va[c][2 * j + 1];
        const T bx = vb[c][2 * j], by = vb[c][2 * j + 1];
        if (k == 0) {
          lds[b * N] = V{ax, bx};
        } else {
          lds[b * N + k] = V{ax - by, ay + bx};
          lds[b * N + N - k] = V{ax + by, bx - ay};
        }
      }
    }
  }
  for (int b = threadIdx.x; b < NB; b += NT) {
    const int64_t r0 = row0 + 2 * b;
    lds[b * N + H] = V{inq[r0].x, inq[r0 + 1].x};
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, +1>(lds, twl);

  constexpr int ITEMS3 = NB * N / RW;
  constexpr int PER3 = (ITEMS3 + NT - 1) / NT;
  double acc = 0.0;
  T* out = a.out + rhs * a.rhs_out;
  T nbar = T(0);
  if constexpr (MODE != ZOUT_REAL) nbar = a.w_scaled ? T(1) : (T)st->nbar;
  const T* wr = a.w + rhs * a.rhs_w;
#pragma unroll
  for (int c = 0; c < PER3; ++c) {
    const int q = threadIdx.x + c * NT;
    if (!(ITEMS3 % NT == 0 || q < ITEMS3)) continue;
    const int b = q / (N / RW), z = (q - b * (N / RW)) * RW;
    const int64_t i0 = (row0 + 2 * b) * N + z, i1 = i0 + N;
    R re, imv;
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const V v = lds[b * N + z + j];
      re[j] = v.x;
      imv[j] = v.y;
    }
    if constexpr (MODE == ZOUT_REAL) {
      const T sc = (T)a.scale;
      st16(out + i0, re * sc);
      st16(out + i1, imv * sc);
    } else if constexpr (MODE == ZOUT_CGQ || MODE == ZOUT_APPLY) {
      const T* p = a.aux + rhs * a.rhs_aux;
      const R p0 = ld16(p + i0), p1 = ld16(p + i1);
      const R w0 = ld16(wr + i0), w1 = ld16(wr + i1);
      const R q0 = re + (nbar * w0) * p0;
      const R q1 = imv + (nbar * w1) * p1;
      st16(out + i0, q0);
      st16(out + i1, q1);
      if constexpr (MODE == ZOUT_CGQ) {
#pragma unroll
        for (int j = 0; j < RW; ++j)
          acc += (double)p0[j] * (double)q0[j] + (double)p1[j] * (double)q1[j];
      }
    } else if constexpr (sizeof(T) == 8) {  // ZOUT_RES: r = b - A x (FP64)
      const T* x = a.aux + rhs * a.rhs_aux;
      const double* bb = a.bvec + rhs * a.rhs_b;
      const R x0 = ld16(x + i0), x1 = ld16(x + i1);
      const R w0 = ld16(wr + i0), w1 = ld16(wr + i1);
      const R r0 = ld16(bb + i0) - (re + (nbar * w0) * x0);
      const R r1 = ld16(bb + i1) - (imv + (nbar * w1) * x1);
      st16(out + i0, r0);
      st16(out + i1, r1);
#pragma unroll
      for (int j = 0; j < RW; ++j) acc += r0[j] * r0[j] + r1[j] * r1[j];
    }
  }
  if constexpr (MODE == ZOUT_CGQ || MODE == ZOUT_RES) {
    const double part = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[(int64_t)rhs * gridDim.x + blockIdx.x] = part;
  }
}

// ---------------------------------------------------------------------------
// z middle pass of the prior-split operator: half spectrum -> real rows ->
// times the noise diagonal -> half spectrum, in place (the rows of a block are
// its own)
// ---------------------------------------------------------------------------
template <typename T, int N, bool RED>
__global__ __launch_bounds__(NT) void k_zmid(ZmidArgs<T> a) {
  using V = cplx<T>;
  using R = vec16<T>;
  constexpr int RW = 16 / sizeof(T);
  constexpr int CW = 16 / sizeof(V);
  constexpr int NB = z_nb<T, N>();
  constexpr int H = N / 2;
  __shared__ __align__(16) V lds[NB * N];
  __shared__ V twl[N];
  const int rhs = blockIdx.y;
  const CgState* st = a.st + rhs;
  if (skip_rhs(st, a.skip)) return;
  const int64_t row0 = (int64_t)blockIdx.x * NB * 2;
  load_twiddles<T, N, NT>(twl, a.tw);
  V* sm = a.spec_main + rhs * a.rhs_main;
  V* sq = a.spec_nyq + rhs * a.rhs_nyq;

  // rows r0, r0 + 1 as Z = A + i B (only the real parts of k = 0 and N/2 enter)
  constexpr int ITEMS = NB * H / CW;
  constexpr int PER = (ITEMS + NT - 1) / NT;
  R va[PER], vb[PER];
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
      const int64_t r0 = row0 + 2 * b;
      va[c] = ld16(reinterpret_cast<const T*>(sm + r0 * H + k0));
      vb[c] = ld16(reinterpret_cast<const T*>(sm + (r0 + 1) * H + k0));
    }
  }
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS % NT == 0 || q < ITEMS) {
      const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        const int k = k0 + j;
        const T ax = va[c][2 * j], ay = va[c][2 * j + 1];
        const T bx = vb[c][2 * j], by = vb[c][2 * j + 1];
        if (k == 0) {
          lds[b * N] = V{ax, bx};
        } else {
          lds[b * N + k] = V{ax - by, ay + bx};
          lds[b * N + N - k] = V{ax + by, bx - ay};
        }
      }
    }
  }
  for (int b = threadIdx.x; b < NB; b += NT) {
    const int64_t r0 = row0 + 2 * b;
    lds[b * N + H] = V{sq[r0].x, sq[r0 + 1].x};
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, +1>(lds, twl);

  // real rows (re: r0, im: r0 + 1) times nbar w; for the folded iteration
  // also the block's sum of nbar w u^2 (its p.q' by Parseval)
  const T nbar = a.w_scaled ? T(1) : (T)st->nbar;
  const T* wr = a.w + rhs * a.rhs_w;
  constexpr int ITEMS3 = NB * N / RW;
  constexpr int PER3 = (ITEMS3 + NT - 1) / NT;
  double wuu = 0.0;  // RED (the folded iteration): the block's sum of nbar w u^2
#pragma unroll
  for (int c = 0; c < PER3; ++c) {
    const int q = threadIdx.x + c * NT;
    if (ITEMS3 % NT == 0 || q < ITEMS3) {
      const int b = q / (N / RW), z = (q - b * (N / RW)) * RW;
      const int64_t i0 = (row0 + 2 * b) * N + z;
      const R w0 = nbar * ld16(wr + i0), w1 = nbar * ld16(wr + i0 + N);
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        const V v = lds[b * N + z + j];
        const V wv = V{v.x * w0[j], v.y * w1[j]};
        lds[b * N + z + j] = wv;
        // FP32 products (relative error 6e-8 each, unbiased), FP64 sums
        if constexpr (RED) wuu += (double)(wv.x * v.x + wv.y * v.y);
      }
    }
  }
  if constexpr (RED) {
    __shared__ double red[NT / 64];
    const double part = block_sum(wuu, red);
    if (threadIdx.x == 0) a.partials[(int64_t)rhs * gridDim.x + blockIdx.x] = part;
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, false, -1>(lds, twl);

  // split the two real rows: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
#pragma unroll
  for (int c = 0; c < PER; ++c) {
    const int q = threadIdx.x + c * NT;
    if (!(ITEMS % NT == 0 || q < ITEMS)) continue;
    const int b = q / (H / CW), k0 = (q - b * (H / CW)) * CW;
    R oa, ob;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int k = k0 + j;
      const V zk = lds[b * N + k];
      const V zn = lds[b * N + ((N - k) % N)];
      oa[2 * j] = T(0.5) * (zk.x + zn.x);
      oa[2 * j + 1] = T(0.5) * (zk.y - zn.y);
      ob[2 * j] = T(0.5) * (zk.y + zn.y);
      ob[2 * j + 1] = T(-0.5) * (zk.x - zn.x);
    }
    const int64_t r0 = row0 + 2 * b;
    st16(reinterpret_cast<T*>(sm + r0 * H + k0), oa);
    st16(reinterpret_cast<T*>(sm + (r0 + 1) * H + k0), ob);
  }
  for (int b = threadIdx.x; b < NB; b += NT) {
    const V zh = lds[b * N + H];
    const int64_t r0 = row0 + 2 * b;
    sq[r0] = V{zh.x, T(0)};
    sq[r0 + 1] = V{zh.y, T(0)};
  }
}

// ---------------------------------------------------------------------------
// strided passes (y or x axis)
// ---------------------------------------------------------------------------
// Layout of the prior-split CG vectors (half spectra touched only by the x
// passes and by pointwise kernels): tile-contiguous in the order the x pass
// reads them.  Column c of outer row o (the columns of an outer row are kz
// for the main part and y for the kz = N/2 plane), x index i:
//   ((o * ncols / TV + c / TV) * N + i) * TV + c % TV,
// TV = the narrower strided tile of the two precisions, so FP32 and FP64
// vectors share the layout.
template <int N> constexpr int vec_tile() {
  return str_tb<float, N>() < str_tb<double, N>() ? str_tb<float, N>() : str_tb<double, N>();
}
template <int N>
__device__ __forceinline__ int64_t vec_off(int outer, int ncols, int c, int i) {
  constexpr int TV = vec_tile<N>();
  return ((int64_t)(outer * (ncols / TV) + c / TV) * N + i) * TV + c % TV;
}

// vec_off as a block's base (columns from c0, a multiple of the layout's tile
// width: the same for every thread) plus the byte offset of column c0 + c, x
// index i from there (below 2^31 for any grid), so that loads and stores can
// take the base from scalar registers and one 32-bit offset per thread.
template <int N>
__device__ __forceinline__ int64_t vec_base(int outer, int ncols, int c0) {
  constexpr int TV = vec_tile<N>();
  return (int64_t)(outer * (ncols / TV) + c0 / TV) * N * TV;
}
template <typename T, int N> __device__ __forceinline__ uint32_t vec_in_bytes(int c, int i) {
  constexpr int TV = vec_tile<N>();
  return (uint32_t)((((c / TV) * N + i) * TV + c % TV) * (int)sizeof(cplx<T>));
}
template <typename T> __device__ __forceinline__ T* at_bytes(T* base, uint32_t bytes) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + bytes);
}
template <typename T> __device__ __forceinline__ const T* at_bytes(const T* base, uint32_t bytes) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + bytes);
}

// Prior-split factor table: c over (|my|, |mx|, kz) in [0, N/2]^3, stored in
// blocks of FB consecutive kz: [|my|][kz / FB][|mx|][kz % FB].  An x-pass
// tile (one |my|, up to FB consecutive kz, every x) then reads one
// contiguous block, and kz pairs load as one aligned vector.
constexpr int FB = SPLIT_FB;
template <int N> constexpr int split_kzb() { return (N / 2 + FB) / FB; }  // kz blocks
template <int N>
__device__ __forceinline__ int64_t fac_off(int my, int mx, int kz) {
  constexpr int H = N / 2 + 1;
  return ((int64_t)(my * split_kzb<N>() + kz / FB) * H + mx) * FB + kz % FB;
}

// Prior-split factors c of the CW elements at x index i, columns cb..cb+CW-1
// of an x-pass segment (its fields give each column's |my| and kz), with the
// kz plane of each and whether it is the monopole.
template <typename T, int N, int CW>
__device__ __forceinline__ void split_facs(const T* __restrict__ fac, const Seg<T>& s, int outer,
                                           int cb, int i, T* f, int* kz, bool* dc) {
  int mx = signed_m(i, N);
  mx = mx < 0 ? -mx : mx;
  if (s.lam_kz < 0) {  // columns are kz = cb + j of the row my = outer
    int my = signed_m(outer, N);
    my = my < 0 ? -my : my;
    const T* row = fac + fac_off<N>(my, mx, cb);  // cb is even: a pair never leaves its block
    if constexpr (CW == 2 && sizeof(T) == 4) {
      const float2 v = *reinterpret_cast<const float2*>(row);
      f[0] = v.x;
      f[1] = v.y;
    } else {
#pragma unroll
      for (int j = 0; j < CW; ++j) f[j] = row[j];
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      kz[j] = cb + j;
      dc[j] = (my | mx | kz[j]) == 0;
    }
  } else {  // columns are my = cb + j of the plane kz = lam_kz
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      int my = signed_m(cb + j, N);
      my = my < 0 ? -my : my;
      kz[j] = s.lam_kz;
      f[j] = fac[fac_off<N>(my, mx, s.lam_kz)];
      dc[j] = false;
    }
  }
}
// sqrt(D) of a kz plane (D = 1 on kz = 0 and kz = N/2, else 2)
template <typename T, int N> __device__ __forceinline__ T sqrt_d(int kz) {
  return (kz == 0 || kz == N / 2) ? T(1) : T(1.41421356237309504880168872420969808);
}

// Output value of the split modes from the forward-transformed element v
// (f: factor, pv: aux value, bv: b value).
template <typename T, int N, int MODE>
__device__ __forceinline__ cplx<T> split_out(T f, int kz, bool dc, cplx<T> v, cplx<T> pv,
                                            cplx<double> bv, double& acc, double& acc2) {
  f *= sqrt_d<T, N>(kz);
  cplx<T> o = {f * v.x, f * v.y};
  if constexpr (MODE == SM_FWD_CGQ) {
    if (!dc) o = cadd(o, pv);
    acc += (double)pv.x * (double)o.x + (double)pv.y * (double)o.y;
  } else if constexpr (MODE == SM_FWD_CGQF) {
    // q' = c sqrt(D) v; pv is p at the monopole only (else zero)
    acc += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
    acc2 += (double)pv.x * (double)o.x + (double)pv.y * (double)o.y;
  } else if constexpr (MODE == SM_FWD_RES) {
    if (!dc) o = cadd(o, pv);
    o = {(T)(bv.x - (double)o.x), (T)(bv.y - (double)o.y)};
    acc += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
  }
  return o;
}

// Waves per SIMD a strided block must allow: its LDS tile (up to 64 KB) fits
// twice per CU, so 1024-thread blocks are held to 64 VGPRs to run two at once.
template <int NTS> constexpr int strided_waves() { return NTS >= 1024 ? 8 : 1; }

template <typename T, int N, int MODE, int TB, int NTS>
__global__ __launch_bounds__(NTS, strided_waves<NTS>()) void k_strided(StrArgs<T> a) {
  constexpr int NT = NTS;
  // nontemporal in the x pass only
  constexpr bool NTA = MODE == SM_FWD_LAM_INV || MODE == SM_INV_SCALE || MODE == SM_INV_DIR ||
                       MODE == SM_FWD_SCALE || MODE == SM_FWD_CGQ || MODE == SM_FWD_RES ||
                       MODE == SM_INV_FOLD || MODE == SM_FWD_CGQF;
  constexpr bool SCALE_IN = MODE == SM_INV_SCALE || MODE == SM_INV_DIR || MODE == SM_INV_FOLD;
  using V = cplx<T>;
  using R = vec16<T>;
  constexpr int CW = 16 / sizeof(V);
  constexpr bool VEC = (TB % CW) == 0;        // TB adjacent columns per row
  constexpr int G = VEC ? CW : 1;             // complex values moved per access
  constexpr int ITEMS = TB * N / G;
  constexpr int PER = (ITEMS + NT - 1) / NT;
  __shared__ __align__(16) V lds[TB * N];
  __shared__ V twl[N];
  constexpr bool SPLIT_OUT = MODE == SM_FWD_SCALE || MODE == SM_FWD_CGQ || MODE == SM_FWD_RES ||
                             MODE == SM_FWD_CGQF;
  constexpr bool REDUCE = MODE == SM_FWD_CGQ || MODE == SM_FWD_RES || MODE == SM_FWD_CGQF;
  __shared__ double red[(REDUCE || MODE == SM_INV_FOLD) ? NT / 64 : 1];
  const int rhs = blockIdx.y;
  if (a.st && skip_rhs(a.st + rhs, a.skip)) return;
  const T* fac_r = a.fac + rhs * a.rhs_fac;
  const T* lam_r = a.lam + rhs * a.rhs_lam;
  int blk = blockIdx.x;
  const bool second = blk >= a.nblk0;
  const Seg<T> s = second ? a.s1 : a.s0;
  if (second) blk -= a.nblk0;
  const int outer = blk / s.n_btiles;
  const int b0 = (blk - outer * s.n_btiles) * TB;

  const V* in = s.in + rhs * s.in_rhs + outer * s.in_outer + b0 * s.in_batch;
  if (!s.axis_contig) {
    // columns b are adjacent in memory (batch stride 1)
    if constexpr (VEC) {
      R buf[PER];
#pragma unroll
      for (int c = 0; c < PER; ++c) {
        const int q = threadIdx.x + c * NT;
        if (ITEMS % NT == 0 || q < ITEMS) {
          const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
          if constexpr (SCALE_IN)
            buf[c] = ld16x<NTA>(at_bytes(reinterpret_cast<const T*>(
                s.in + rhs * s.in_rhs + vec_base<N>(outer, s.n_btiles * TB, b0)),
                vec_in_bytes<T, N>(b, i)));
          else
            buf[c] = ld16x<NTA>(reinterpret_cast<const T*>(in + i * s.in_axis + b));
        }
      }
      if constexpr (MODE == SM_INV_DIR) {
        // CG direction: `in` is r; the pending x += alpha p, then p = r + beta p
        const CgState* cs = a.st + rhs;
        const bool first = cs->first != 0, pending = cs->pending != 0;
        const T alpha = (T)cs->alpha, beta = (T)cs->beta;
        const int64_t vb = rhs * s.in_rhs + vec_base<N>(outer, s.n_btiles * TB, b0);
        T* pb = reinterpret_cast<T*>(s.p + vb);
        T* xb = reinterpret_cast<T*>(s.x + vb);
#pragma unroll
        for (int c = 0; c < PER; ++c) {
          const int q = threadIdx.x + c * NT;
          if (ITEMS % NT == 0 || q < ITEMS) {
            const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
            const uint32_t vo = vec_in_bytes<T, N>(b, i);
            T* pp = at_bytes(pb, vo);
            if (!first) {
              const R pv = ld16x<NTA>(pp);
              if (pending) {
                T* xp = at_bytes(xb, vo);
                st16x<NTA>(xp, ld16x<NTA>(xp) + alpha * pv);
              }
              buf[c] += beta * pv;
            }
            st16x<NTA>(pp, buf[c]);
          }
        }
      }
      // scaled (SCALE_IN) into the LDS tile.  INV_FOLD also sums |p|^2 of the
      // group's reals from index pp_from on (0: all, 2: without the monopole;
      // the default, one past the last, none) here, where the values are read
      // anyway: summed in the direction loops, it made the pass spill
      // registers under its 64-VGPR cap
      double ppn = 0.0;
      auto to_lds = [&](int c, int pp_from = 16 / (int)sizeof(T)) {
        const int q = threadIdx.x + c * NT;
        if constexpr (MODE == SM_INV_FOLD) {
          T sq = T(0);  // (FP32 over the group's four values: fewer registers)
#pragma unroll
          for (int j = 0; j < 2 * CW; ++j)
            if (j >= pp_from) sq += buf[c][j] * buf[c][j];
          ppn += (double)sq;
        }
        if constexpr (SCALE_IN) {
          const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
          T f[CW];
          int kz[CW];
          bool dc[CW];
          split_facs<T, N, CW>(fac_r, s, outer, b0 + b, i, f, kz, dc);
#pragma unroll
          for (int j = 0; j < CW; ++j) {
            const T g = f[j] * ((T)a.in_scale / sqrt_d<T, N>(kz[j]));
            buf[c][2 * j] *= g;
            buf[c][2 * j + 1] *= g;
          }
        }
        *reinterpret_cast<R*>(lds + q * CW) = buf[c];
      };
      if constexpr (MODE == SM_INV_FOLD) {
        // folded CG step: `in` is r and `q` holds q', the noise part of the
        // previous A p.  Pending (the previous iteration's alpha and beta):
        // x += alpha p, r -= alpha ([m != 0] p + q'), p = r + beta p.  First
        // direction of a cycle: p = r.  Otherwise p is ready (a reliable
        // update continued it).  Block partials of the new r.r and of p.p
        // without the monopole.
        const CgState* cs = a.st + rhs;
        const bool pending = cs->pending != 0, first = cs->first != 0;
        const T alpha = (T)cs->alpha, beta = (T)cs->beta;
        // the monopole is element 0 of column 0, row 0, outer row 0 (main part)
        const bool dc_tile = s.lam_kz < 0 && outer == 0 && b0 == 0;
        const int64_t vb = rhs * s.in_rhs + vec_base<N>(outer, s.n_btiles * TB, b0);
        T* pb = reinterpret_cast<T*>(s.p + vb);
        T* xb = reinterpret_cast<T*>(s.x + vb);
        T* rb = reinterpret_cast<T*>(s.r + vb);
        const T* qb = reinterpret_cast<const T*>(s.q + vb);
        double rr = 0.0;
        if (pending) {
          // one element group at a time (few registers: two blocks per CU)
#pragma unroll
          for (int c = 0; c < PER; ++c) {
            const int q = threadIdx.x + c * NT;
            if (ITEMS % NT == 0 || q < ITEMS) {
              const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
              const uint32_t vo = vec_in_bytes<T, N>(b, i);
              const R pv = ld16x<NTA>(at_bytes(pb, vo));
              const R qv = ld16x<NTA>(at_bytes(qb, vo));
              const R xv = ld16x<NTA>(at_bytes(xb, vo));
              st16x<NTA>(at_bytes(xb, vo), xv + alpha * pv);
              R qe = qv + pv;
              const bool dc0 = c == 0 && dc_tile && q == 0;  // (i, b) = (0, 0)
              if (dc0) {
                qe[0] = qv[0];
                qe[1] = qv[1];
              }
              const R rn = buf[c] - alpha * qe;
              st16x<NTA>(at_bytes(rb, vo), rn);
#pragma unroll
              for (int j = 0; j < 2 * CW; ++j) rr += (double)rn[j] * (double)rn[j];
              buf[c] = rn + beta * pv;
              st16x<NTA>(at_bytes(pb, vo), buf[c]);
              to_lds(c, dc0 ? 2 : 0);
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < PER; ++c) {
            const int q = threadIdx.x + c * NT;
            if (ITEMS % NT == 0 || q < ITEMS) {
              const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
#pragma unroll
              for (int j = 0; j < 2 * CW; ++j) rr += (double)buf[c][j] * (double)buf[c][j];
              T* pp = at_bytes(pb, vec_in_bytes<T, N>(b, i));
              if (first) st16x<NTA>(pp, buf[c]);
              else buf[c] = ld16x<NTA>(pp);
              const bool dc0 = c == 0 && dc_tile && q == 0;  // (i, b) = (0, 0)
              to_lds(c, dc0 ? 2 : 0);
            }
          }
        }
        const double part = block_sum(rr, red);
        const double part2 = block_sum(ppn, red);
        if (threadIdx.x == 0) {
          a.partials[(int64_t)rhs * 2 * gridDim.x + blockIdx.x] = part;
          a.partials[((int64_t)rhs * 2 + 1) * gridDim.x + blockIdx.x] = part2;
        }
      } else {
#pragma unroll
        for (int c = 0; c < PER; ++c) {
          const int q = threadIdx.x + c * NT;
          if (ITEMS % NT == 0 || q < ITEMS) to_lds(c);
        }
      }
    } else {
      double rr_nv = 0.0, pp_nv = 0.0;  // INV_FOLD: r.r and p.p of this thread
      for (int e = threadIdx.x; e < TB * N; e += NT) {
        const int b = e % TB, i = e / TB;
        V v;
        if constexpr (SCALE_IN) v = s.in[rhs * s.in_rhs + vec_off<N>(outer, s.n_btiles * TB, b0 + b, i)];
        else v = in[i * s.in_axis + b];
        if constexpr (MODE == SM_INV_DIR) {
          const CgState* cs = a.st + rhs;
          const int64_t o = rhs * s.in_rhs + vec_off<N>(outer, s.n_btiles * TB, b0 + b, i);
          if (!cs->first) {
            const V pv = s.p[o];
            if (cs->pending) {
              const T al = (T)cs->alpha;
              s.x[o] = V{s.x[o].x + al * pv.x, s.x[o].y + al * pv.y};
            }
            const T be = (T)cs->beta;
            v = V{v.x + be * pv.x, v.y + be * pv.y};
          }
          s.p[o] = v;
        }
        if constexpr (MODE == SM_INV_FOLD) {
          const CgState* cs = a.st + rhs;
          const int64_t o = rhs * s.in_rhs + vec_off<N>(outer, s.n_btiles * TB, b0 + b, i);
          const bool dc = s.lam_kz < 0 && outer == 0 && b0 + b == 0 && i == 0;
          if (cs->pending) {
            const T al = (T)cs->alpha, be = (T)cs->beta;
            const V pv = s.p[o], qv = s.q[o], xv = s.x[o];
            s.x[o] = V{xv.x + al * pv.x, xv.y + al * pv.y};
            const V qe = dc ? qv : V{qv.x + pv.x, qv.y + pv.y};
            v = V{v.x - al * qe.x, v.y - al * qe.y};
            s.r[o] = v;
            rr_nv += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            v = V{v.x + be * pv.x, v.y + be * pv.y};
            s.p[o] = v;
          } else {
            rr_nv += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            if (cs->first) s.p[o] = v;
            else v = s.p[o];
          }
          if (!dc) pp_nv += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
        if constexpr (SCALE_IN) {
          T f;
          int kz;
          bool dc;
          split_facs<T, N, 1>(fac_r, s, outer, b0 + b, i, &f, &kz, &dc);
          f *= (T)a.in_scale / sqrt_d<T, N>(kz);
          v = {v.x * f, v.y * f};
        }
        lds[e] = v;
      }
      if constexpr (MODE == SM_INV_FOLD) {
        const double part = block_sum(rr_nv, red);
        const double part2 = block_sum(pp_nv, red);
        if (threadIdx.x == 0) {
          a.partials[(int64_t)rhs * 2 * gridDim.x + blockIdx.x] = part;
          a.partials[((int64_t)rhs * 2 + 1) * gridDim.x + blockIdx.x] = part2;
        }
      }
    }
  } else {
    // the FFT axis is contiguous (batch stride s.in_batch)
    constexpr int AV = (N % CW == 0) ? CW : 1;
    constexpr int IT = TB * N / AV;
    constexpr int PA = (IT + NT - 1) / NT;
    V buf[PA][AV];
#pragma unroll
    for (int c = 0; c < PA; ++c) {
      const int q = threadIdx.x + c * NT;
      if (IT % NT == 0 || q < IT) {
        const int b = q / (N / AV), i = (q - b * (N / AV)) * AV;
        if constexpr (AV == CW && CW > 1) {
          const R v = ld16x<NTA>(reinterpret_cast<const T*>(in + b * s.in_batch + i));
#pragma unroll
          for (int j = 0; j < AV; ++j) buf[c][j] = V{v[2 * j], v[2 * j + 1]};
        } else {
          buf[c][0] = in[b * s.in_batch + i];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < PA; ++c) {
      const int q = threadIdx.x + c * NT;
      if (IT % NT == 0 || q < IT) {
        const int b = q / (N / AV), i = (q - b * (N / AV)) * AV;
#pragma unroll
        for (int j = 0; j < AV; ++j) lds[(i + j) * TB + b] = buf[c][j];
      }
    }
  }
  load_twiddles<T, N, NT>(twl, a.tw);
  // split CGQ / RES: the aux vector and the prior-split factors at the
  // output's positions, requested before the FFT so that the loads complete
  // under it (VEC tiles of up to 512 threads; with 1024 the registers are
  // short and other waves hide the loads, issued after the FFT).  Measured at
  // 512^3: the factors read here instead of after the FFT make the x forward
  // with q 7 % faster.
  // (the folded iteration's x forward reads no aux vector)
  constexpr bool PRELOAD = REDUCE && VEC && NT <= 512;
  constexpr bool PRE_AUX = PRELOAD && MODE != SM_FWD_CGQF;
  // the split output's tile in the vector layout, and the aux vector's
  const int64_t vb_out = rhs * s.out_rhs + vec_base<N>(outer, s.n_btiles * TB, b0);
  const T* auxb = REDUCE ? reinterpret_cast<const T*>(s.aux + vb_out) : nullptr;
  R avp[PRE_AUX ? PER : 1];
  T fpre[PRELOAD ? PER : 1][CW];
  if constexpr (PRELOAD) {
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int q = threadIdx.x + c * NT;
      if (ITEMS % NT == 0 || q < ITEMS) {
        const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
        if constexpr (PRE_AUX) avp[c] = ld16x<NTA>(at_bytes(auxb, vec_in_bytes<T, N>(b, i)));
        int kzp[CW];
        bool dcp[CW];
        split_facs<T, N, CW>(fac_r, s, outer, b0 + b, i, fpre[c], kzp, dcp);
      }
    }
  }
  if constexpr (MODE == SM_FWD_LAM_INV) {
    // Lambda of the elements this thread holds between the forward and the
    // inverse transform, read from the column's row of the x-pass table
    // before the forward FFT so that the loads complete under it.  Row
    // (|my|, kz) holds tuples A_t[k] = Lambda(my^2 + kz^2 + (t + k L)^2),
    // t = 0..L, k < R/2 (L = N/R, R the last radix).  The butterfly j holds
    // elements e = j + r L: |m| = j + r L for r < R/2, and
    // (L - j) + (R - 1 - r) L for the others, i.e. A_j and A_(L-j) reversed.
    constexpr int RL = last_radix<N>();
    static_assert(RL % 2 == 0, "x pass needs an even last radix");
    constexpr int HR = RL / 2;
    constexpr int L = N / RL;
    constexpr int HN = N / 2 + 1;
    constexpr int ROW = (L + 1) * HR;
    constexpr int NBF = TB * L;
    constexpr int PL = (NBF + NT - 1) / NT;
    T lamv[PL][RL];
    const int my_o = s.lam_y_outer ? signed_m(outer, N) : 0;
#pragma unroll
    for (int c = 0; c < PL; ++c) {
      const int bf = threadIdx.x + c * NT;
      if (NBF % NT == 0 || bf < NBF) {
        const int b = bf % TB, j = bf / TB, cb = b0 + b;
        const int my = s.lam_y_outer ? my_o : signed_m(cb, N);
        const int kz = s.lam_kz < 0 ? cb : s.lam_kz;
        const T* row = lam_r + (int64_t)((my < 0 ? -my : my) * HN + kz) * ROW;
        const T* lo = row + j * HR;
        const T* hi = row + (L - j) * HR;
        if constexpr ((HR * sizeof(T)) % 16 == 0) {
          constexpr int VW = 16 / sizeof(T);
#pragma unroll
          for (int v = 0; v < HR / VW; ++v) {
            const vec16<T> x0 = *reinterpret_cast<const vec16<T>*>(lo + v * VW);
            const vec16<T> x1 = *reinterpret_cast<const vec16<T>*>(hi + v * VW);
#pragma unroll
            for (int k = 0; k < VW; ++k) {
              lamv[c][v * VW + k] = x0[k];
              lamv[c][RL - 1 - (v * VW + k)] = x1[k];
            }
          }
        } else {
#pragma unroll
          for (int k = 0; k < HR; ++k) {
            lamv[c][k] = lo[k];
            lamv[c][RL - 1 - k] = hi[k];
          }
        }
      }
    }
    __syncthreads();
    fft_tile_diag<T, N, TB, NT>(lds, twl, lamv);
  } else {
    __syncthreads();
    if constexpr (MODE == SM_INV || SCALE_IN) fft_tile<T, N, TB, NT, true, +1>(lds, twl);
    else fft_tile<T, N, TB, NT, true, -1>(lds, twl);
  }

  V* out = s.out + rhs * s.out_rhs + outer * s.out_outer + b0 * s.out_batch;
  if constexpr (MODE == SM_FWD_CROP) {
    const int no = s.n_out, h = no / 2;
    for (int e = threadIdx.x; e < TB * no; e += NT) {
      const int b = e % TB, o = e / TB;
      V v = {T(0), T(0)};
      if (o != h) v = lds[(o < h ? o : o + (N - no)) * TB + b];
      out[o * s.out_axis + b] = v;
    }
  } else if constexpr (SPLIT_OUT) {
    // x-pass segments only (the batch is contiguous)
    double acc = 0.0, acc2 = 0.0;
    const int64_t ob = rhs * s.out_rhs;
    const int ncols = s.n_btiles * TB;
    if constexpr (VEC) {
#pragma unroll
      for (int c = 0; c < PER; ++c) {
        const int q = threadIdx.x + c * NT;
        if (ITEMS % NT == 0 || q < ITEMS) {
          const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
          const uint32_t vo = vec_in_bytes<T, N>(b, i);
          const R v = *reinterpret_cast<const R*>(lds + q * CW);
          R av{};
          if constexpr (PRE_AUX) {
            av = avp[c];
          } else if constexpr (REDUCE && MODE != SM_FWD_CGQF) {
            av = ld16x<NTA>(at_bytes(auxb, vo));
          }
          T f[CW];
          int kz[CW];
          bool dc[CW];
          split_facs<T, N, CW>(fac_r, s, outer, b0 + b, i, f, kz, dc);
          if constexpr (MODE == SM_FWD_CGQF) {
#pragma unroll
            for (int j = 0; j < CW; ++j)
              if (dc[j]) {
                const cplx<T> p0 =
                    *reinterpret_cast<const cplx<T>*>(at_bytes(auxb, vo + j * (uint32_t)sizeof(V)));
                av[2 * j] = p0.x;
                av[2 * j + 1] = p0.y;
              }
          }
          if constexpr (PRELOAD) {
#pragma unroll
            for (int j = 0; j < CW; ++j) f[j] = fpre[c][j];  // (the loads above fold away)
          }
          R o;
#pragma unroll
          for (int j = 0; j < CW; ++j) {
            cplx<double> bv{0.0, 0.0};
            if constexpr (MODE == SM_FWD_RES) bv = s.bvec[vb_out + vo / sizeof(V) + j];
            const cplx<T> r = split_out<T, N, MODE>(f[j], kz[j], dc[j], V{v[2 * j], v[2 * j + 1]},
                                                    V{av[2 * j], av[2 * j + 1]}, bv, acc, acc2);
            o[2 * j] = r.x;
            o[2 * j + 1] = r.y;
          }
          st16x<NTA>(at_bytes(reinterpret_cast<T*>(s.out + vb_out), vo), o);
        }
      }
    } else {
      for (int e = threadIdx.x; e < TB * N; e += NT) {
        const int b = e % TB, i = e / TB;
        const int64_t off = ob + vec_off<N>(outer, ncols, b0 + b, i);
        T f;
        int kz;
        bool dc;
        split_facs<T, N, 1>(fac_r, s, outer, b0 + b, i, &f, &kz, &dc);
        const V pv = (REDUCE && (MODE != SM_FWD_CGQF || dc)) ? s.aux[off] : V{T(0), T(0)};
        cplx<double> bv{0.0, 0.0};
        if constexpr (MODE == SM_FWD_RES) bv = s.bvec[off];
        s.out[off] = split_out<T, N, MODE>(f, kz, dc, lds[e], pv, bv, acc, acc2);
      }
    }
    if constexpr (MODE == SM_FWD_CGQF) {
      const double part = block_sum(acc, red);
      const double part2 = block_sum(acc2, red);
      if (threadIdx.x == 0) {
        a.partials[(int64_t)rhs * 2 * gridDim.x + blockIdx.x] = part;
        a.partials[((int64_t)rhs * 2 + 1) * gridDim.x + blockIdx.x] = part2;
      }
    } else if constexpr (REDUCE) {
      const double part = block_sum(acc, red);
      if (threadIdx.x == 0) a.partials[(int64_t)rhs * gridDim.x + blockIdx.x] = part;
    }
  } else if (!s.axis_contig) {
    if constexpr (VEC) {
#pragma unroll
      for (int c = 0; c < PER; ++c) {
        const int q = threadIdx.x + c * NT;
        if (ITEMS % NT == 0 || q < ITEMS) {
          const int i = q / (TB / CW), b = (q - i * (TB / CW)) * CW;
          // the FP32 x inverse writes its spectrum with cached stores (the y
          // pass reads it next): measured at 512^3 the folded x inverse is
          // 32 us faster and the y pass 14 us slower than with nontemporal
          // stores; in FP64 both are slower, and keep nontemporal ones
          st16x<NTA && !(SCALE_IN && sizeof(T) == 4)>(
              reinterpret_cast<T*>(out + i * s.out_axis + b), *reinterpret_cast<const R*>(lds + q * CW));
        }
      }
    } else {
      for (int e = threadIdx.x; e < TB * N; e += NT) {
        const int b = e % TB, i = e / TB;
        out[i * s.out_axis + b] = lds[e];
      }
    }
  } else {
    constexpr int AV = (N % CW == 0) ? CW : 1;
    constexpr int IT = TB * N / AV;
    for (int q = threadIdx.x; q < IT; q += NT) {
      const int b = q / (N / AV), i = (q - b * (N / AV)) * AV;
      if constexpr (AV == CW && CW > 1) {
        R v;
#pragma unroll
        for (int j = 0; j < AV; ++j) {
          const V x = lds[(i + j) * TB + b];
          v[2 * j] = x.x;
          v[2 * j + 1] = x.y;
        }
        st16x<NTA>(reinterpret_cast<T*>(out + b * s.out_batch + i), v);
      } else {
        out[b * s.out_batch + i] = lds[i * TB + b];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// finalize: sum the block partials of one reduction per RHS (fixed order)
// and update the scalar CG state
// ---------------------------------------------------------------------------
// The finalize kernels run one block per RHS.  Their sums of block partials
// (tens of thousands, in L2) are bound by load round trips: each thread keeps
// eight independent loads in flight per round, summed in a fixed order.
constexpr int FIN_THREADS = 1024;
__device__ __forceinline__ double sum_parts(const double* p, int nparts, double* red) {
  constexpr int U = 8;
  double s[U];
#pragma unroll
  for (int u = 0; u < U; ++u) s[u] = 0.0;
  int i = threadIdx.x;
  for (; i + (U - 1) * FIN_THREADS < nparts; i += U * FIN_THREADS) {
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] += p[i + u * FIN_THREADS];
  }
  for (; i < nparts; i += FIN_THREADS) s[0] += p[i];
  const double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  return block_sum(t, red);
}

// Iteration bookkeeping and stopping once the new recursive residual r.r is
// known (thread 0).
__device__ __forceinline__ void count_iteration(CgState* st, double rho_new) {
  st->iter += 1;
  const double rel = sqrt(rho_new) / st->bnorm;
  st->rel = rel;
  if (st->reliable) {
    // the recursive residual decides when to refresh it in FP64; only the
    // FP64 residual decides convergence
    // (while holding for the solution to settle only the drop by delta
    // triggers); an interval longer than three times the mean so far ends
    // too, so that a solve at its attainable accuracy, whose FP32 residual
    // hardly falls any more, reaches its stagnation test
    const int32_t mean = st->updates > 0 ? st->upd_iter / st->updates : 0;
    const bool long_interval = st->updates > 0 && st->iter - st->upd_iter > 3 * mean + 10;
    if (sqrt(rho_new) <= st->delta * st->rmax || (rel <= st->tol && !st->hold) ||
        st->iter >= st->max_iter || long_interval) {
      st->done = 1;
      st->status = CG_UPDATE;
    }
  } else if (rel <= st->tol) {
    st->done = 1;
    st->status = CG_CONVERGED;
  } else if (st->iter >= st->max_iter) {
    st->done = 1;
    st->status = CG_MAXITER;
  }
}

template <int KIND>
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double* partials, int nparts,
                                                          int skip, CgState* st_all) {
  __shared__ double red[FIN_THREADS / 64];
  const int rhs = blockIdx.x;
  CgState* st = st_all + rhs;
  if (skip_rhs(st, skip)) return;
  if constexpr (KIND == FIN_RRF) {
    // after INV_FOLD: the new r.r and p.p (two regions); when the pass
    // applied the previous step, one iteration more
    const double* p = partials + (int64_t)rhs * 2 * nparts;
    const double tot = sum_parts(p, nparts, red);
    const double ppn = sum_parts(p + nparts, nparts, red);
    if (threadIdx.x != 0) return;
    if (st->pending) {
      count_iteration(st, tot);
      st->rho_old = st->rho;
    }
    st->rho = tot;
    st->pp = ppn;
    st->first = 0;
    st->pending = 0;
    return;
  } else {
    const double tot = sum_parts(partials + (int64_t)rhs * nparts, nparts, red);
    if (threadIdx.x != 0) return;
    if constexpr (KIND == FIN_PQ) {
      st->pending = 0;  // the z pass of this iteration applied it
      st->pq = tot;
      if (!(tot > 0.0) || !isfinite(tot)) {
        st->done = 1;
        st->status = CG_BREAKDOWN;
      } else {
        st->alpha = st->rho / tot;
      }
    } else if constexpr (KIND == FIN_RR) {
      count_iteration(st, tot);
      st->beta = tot / st->rho;
      st->rho_old = st->rho;
      st->rho = tot;
      st->first = 0;
      st->pending = 1;
    } else {  // FIN_RES
      st->outer_rr = tot;
    }
  }
}

// Folded iteration, after FWD_CGQF: p.q and q.q from p.p (FIN_RRF), the z
// middle pass's sums of nbar w u^2 and FWD_CGQF's q'.q' and monopole term;
// alpha, and beta from the recurrence.
__global__ __launch_bounds__(FIN_THREADS) void k_finalize_fold_pq(const double* part_z, int nzb,
                                                          const double* part_x, int nxb,
                                                          double m_cells, int skip,
                                                          CgState* st_all) {
  __shared__ double red[FIN_THREADS / 64];
  const int rhs = blockIdx.x;
  CgState* st = st_all + rhs;
  if (skip_rhs(st, skip)) return;
  const double wuu = sum_parts(part_z + (int64_t)rhs * nzb, nzb, red);
  const double* px = part_x + (int64_t)rhs * 2 * nxb;
  const double qnqn = sum_parts(px, nxb, red);
  const double p0q0 = sum_parts(px + nxb, nxb, red);
  if (threadIdx.x != 0) return;
  // q = [m != 0] p + q' with p.q' = M sum(nbar w u^2) (Parseval: q' is
  // C diag(nbar w) C p in the half-spectrum inner product)
  const double pqn = m_cells * wuu;
  const double pq = st->pp + pqn;
  const double qq = st->pp + 2.0 * (pqn - p0q0) + qnqn;
  st->pq = pq;
  if (!(pq > 0.0) || !isfinite(pq)) {
    st->done = 1;
    st->status = CG_BREAKDOWN;
    st->pending = 0;
    return;
  }
  // alpha from the exact r.r; the next r.r for beta before r itself is
  // updated: |r - alpha q|^2 = r.r - 2 alpha r.q + alpha^2 q.q, with r.q =
  // p.q (r and p differ by a multiple of the previous direction, which is
  // conjugate to p), that is alpha^2 q.q - r.r.  A negative value (total
  // cancellation) restarts the direction.
  const double alpha = st->rho / pq;
  const double rho_next = alpha * alpha * qq - st->rho;
  st->alpha = alpha;
  st->beta = rho_next > 0.0 ? rho_next / st->rho : 0.0;
  st->pending = 1;
}

hipError_t launch_finalize_fold_pq(const double* part_z, int nzb, const double* part_x, int nxb,
                                   double m_cells, int skip, CgState* st, int nrhs,
                                   hipStream_t s) {
  klaunch(k_finalize_fold_pq, dim3(nrhs), dim3(FIN_THREADS), 0, s, part_z, nzb, part_x, nxb,
          m_cells, skip, st);
  return hipGetLastError();
}

hipError_t launch_finalize(int kind, const double* partials, int nparts, int skip, CgState* st,
                           int nrhs, hipStream_t s) {
  switch (kind) {
    case FIN_PQ:
      klaunch(k_finalize<FIN_PQ>, dim3(nrhs), dim3(FIN_THREADS), 0, s, partials, nparts, skip, st);
      break;
    case FIN_RR:
      klaunch(k_finalize<FIN_RR>, dim3(nrhs), dim3(FIN_THREADS), 0, s, partials, nparts, skip, st);
      break;
    case FIN_RES:
      klaunch(k_finalize<FIN_RES>, dim3(nrhs), dim3(FIN_THREADS), 0, s, partials, nparts, skip, st);
      break;
    case FIN_RRF:
      klaunch(k_finalize<FIN_RRF>, dim3(nrhs), dim3(FIN_THREADS), 0, s, partials, nparts, skip, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// x-pass Lambda rows: for every column (|my|, kz) of the half spectrum, the
// diagonal of eq:WF at the moduli the x pass holds in its fused stage, laid
// out so that each thread reads two contiguous tuples (see k_strided)
// ---------------------------------------------------------------------------
template <int N> constexpr int64_t xlam_row() {
  return (int64_t)(N / last_radix<N>() + 1) * (last_radix<N>() / 2);
}

template <int N>
__global__ void k_xlam_rows(const double* __restrict__ lam, double* rows64, float* rows32) {
  constexpr int HR = last_radix<N>() / 2, L = N / last_radix<N>(), HN = N / 2 + 1;
  constexpr int64_t ROW = xlam_row<N>();
  const int64_t total = (int64_t)HN * HN * ROW;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t col = i / ROW;
    const int pos = (int)(i - col * ROW);
    const int my = (int)(col / HN), kz = (int)(col - (int64_t)my * HN);
    const int t = pos / HR, k = pos - t * HR;
    const int mx = t + k * L;  // <= N/2
    const double v = lam[(int64_t)my * my + (int64_t)kz * kz + (int64_t)mx * mx];
    rows64[i] = v;
    rows32[i] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// launchers (dispatch over the supported lengths)
// ---------------------------------------------------------------------------
#define WF_FOR_LENGTHS(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
// FP32 kernels are only instantiated for target grids (<= 512).
#define WF_FOR_F32(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

bool fft_length_supported(int n, bool fp64) {
  switch (n) {
#define X(L) case L:
    WF_FOR_LENGTHS(X)
#undef X
    return fp64 || n <= 512;
    default: return false;
  }
}

int64_t split_fac_elems(int n) {
  const int64_t h = n / 2 + 1, kzb = (n / 2 + FB) / FB;
  return (n >= 8 && n % 2 == 0) ? h * kzb * h * FB : 0;
}

// i = ((my * kzb + kb) * h + mx) * FB + kr, kz = kb * FB + kr
__global__ void k_split_fac(const double* __restrict__ lam, int h, int kzb, double m_cells,
                            double* fac64, float* fac32) {
  const int64_t total = (int64_t)h * kzb * h * FB;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int kr = (int)(i % FB);
    const int64_t r1 = i / FB;
    const int mx = (int)(r1 % h);
    const int64_t r2 = r1 / h;
    const int kb = (int)(r2 % kzb), my = (int)(r2 / kzb);
    const int kz = kb * FB + kr;
    double c = 0.0;  // padding
    if (kz < h) {
      int64_t j = (int64_t)my * my + (int64_t)mx * mx + (int64_t)kz * kz;
      if (j == 0) j = 1;  // the monopole takes the |m|^2 = 1 value
      c = 1.0 / sqrt(lam[j] * m_cells);
    }
    fac64[i] = c;
    fac32[i] = (float)c;
  }
}

hipError_t launch_split_fac(int n, const double* lam, double m_cells, double* fac64, float* fac32,
                            hipStream_t s) {
  const int64_t total = split_fac_elems(n);
  if (total <= 0) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  klaunch(k_split_fac, dim3(blocks), dim3(256), 0, s, lam, n / 2 + 1,
                     (n / 2 + FB) / FB, m_cells, fac64, fac32);
  return hipGetLastError();
}

int64_t xlam_elems(int n) {
  switch (n) {
#define X(L) \
  case L: return (int64_t)(L / 2 + 1) * (L / 2 + 1) * xlam_row<L>();
    WF_FOR_F32(X)
#undef X
    default: return 0;
  }
}

hipError_t launch_xlam_rows(int n, const double* lam, double* rows64, float* rows32,
                            hipStream_t s) {
  const int64_t total = xlam_elems(n);
  if (total <= 0) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  switch (n) {
#define X(L) \
  case L: klaunch(k_xlam_rows<L>, dim3(blocks), dim3(256), 0, s, lam, rows64, rows32); break;
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Strided tiles: TB = str_tb<T, N> adjacent columns, 512 threads (1024 for
// some FP32 passes, see strided_n).
constexpr int NT_STRIDED = 512;

int strided_tb(int n, bool fp64) {
  switch (n) {
#define X(L) \
  case L: return fp64 ? str_tb<double, L>() : str_tb<float, L>();
    WF_FOR_LENGTHS(X)
#undef X
    default: return 0;
  }
}

int split_vec_tile(int n) {
  switch (n) {
#define X(L) \
  case L: return vec_tile<L>();
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

int zpass_blocks(int n, int64_t nrows, bool fp64) { return (int)(nrows / (2 * zpass_nb(n, fp64))); }

template <typename T, int N>
static hipError_t zfwd_n(int mode, const ZfwdArgs<T>& a, int64_t nrows, int nrhs, hipStream_t s) {
  constexpr int NB = z_nb<T, N>();
  dim3 grid((unsigned)(nrows / (2 * NB)), (unsigned)nrhs);
  switch (mode) {
    case ZIN_REAL: klaunch((k_zfwd<T, N, ZIN_REAL>), grid, dim3(NT), 0, s, a); break;
    case ZIN_CGP: klaunch((k_zfwd<T, N, ZIN_CGP>), grid, dim3(NT), 0, s, a); break;
    case ZIN_I64:
      if constexpr (sizeof(T) == 8) {
        klaunch((k_zfwd<T, N, ZIN_I64>), grid, dim3(NT), 0, s, a);
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
    case ZOUT_REAL: klaunch((k_zinv<T, N, ZOUT_REAL>), grid, dim3(NT), 0, s, a); break;
    case ZOUT_CGQ: klaunch((k_zinv<T, N, ZOUT_CGQ>), grid, dim3(NT), 0, s, a); break;
    case ZOUT_RES:
      if constexpr (sizeof(T) == 8) {
        klaunch((k_zinv<T, N, ZOUT_RES>), grid, dim3(NT), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case ZOUT_APPLY: klaunch((k_zinv<T, N, ZOUT_APPLY>), grid, dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t zmid_n(const ZmidArgs<T>& a, int64_t nrows, int nrhs, hipStream_t s) {
  constexpr int NB = z_nb<T, N>();
  dim3 grid((unsigned)(nrows / (2 * NB)), (unsigned)nrhs);
  if constexpr (sizeof(T) == 4) {
    if (a.partials) {
      klaunch((k_zmid<T, N, true>), grid, dim3(NT), 0, s, a);
      return hipGetLastError();
    }
  } else {
    if (a.partials) return hipErrorInvalidValue;  // the folded iteration is FP32 only
  }
  klaunch((k_zmid<T, N, false>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N, int TBV, int NTV>
static hipError_t strided_v(int mode, const StrArgs<T>& a, int nrhs, hipStream_t s) {
  dim3 grid((unsigned)(a.nblk0 + a.nblk1), (unsigned)nrhs);
  switch (mode) {
    case SM_FWD: klaunch((k_strided<T, N, SM_FWD, TBV, NTV>), grid, dim3(NTV), 0, s, a); break;
    case SM_INV: klaunch((k_strided<T, N, SM_INV, TBV, NTV>), grid, dim3(NTV), 0, s, a); break;
    case SM_FWD_LAM_INV:
      klaunch((k_strided<T, N, SM_FWD_LAM_INV, TBV, NTV>), grid, dim3(NTV), 0, s, a);
      break;
    case SM_FWD_CROP:
      klaunch((k_strided<T, N, SM_FWD_CROP, TBV, NTV>), grid, dim3(NTV), 0, s, a);
      break;
    case SM_INV_FOLD:
    case SM_FWD_CGQF:
      // the folded iteration exists for FP32 vectors only
      if constexpr (sizeof(T) == 4) {
        if (mode == SM_INV_FOLD)
          klaunch((k_strided<T, N, SM_INV_FOLD, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else
          klaunch((k_strided<T, N, SM_FWD_CGQF, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    case SM_INV_SCALE:
    case SM_INV_DIR:
    case SM_FWD_SCALE:
    case SM_FWD_CGQ:
    case SM_FWD_RES:
      if constexpr (N <= 512) {
        if (mode == SM_INV_SCALE)
          klaunch((k_strided<T, N, SM_INV_SCALE, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else if (mode == SM_INV_DIR)
          klaunch((k_strided<T, N, SM_INV_DIR, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else if (mode == SM_FWD_SCALE)
          klaunch((k_strided<T, N, SM_FWD_SCALE, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else if (mode == SM_FWD_CGQ)
          klaunch((k_strided<T, N, SM_FWD_CGQ, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else if constexpr (sizeof(T) == 8)
          klaunch((k_strided<T, N, SM_FWD_RES, TBV, NTV>), grid, dim3(NTV), 0, s, a);
        else
          return hipErrorInvalidValue;
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Tiles of the large grids run 1024 threads (half the loads per thread and
// array, two blocks of 16 waves per CU instead of two of 8).  Measured at
// 512^3: FP32, the y passes and the x inverse with the CG direction are
// 3-4 % faster, the x forward with q is slower (its 1024-thread form spills
// under the 64-VGPR cap) and keeps 512; FP64, the y passes and the plain x
// pass are 3-4 % faster, the x passes of the split CG (direction, q,
// residual) are not and keep 512.
template <typename T, int N>
static hipError_t strided_n(int mode, const StrArgs<T>& a, int nrhs, hipStream_t s) {
  if constexpr (N >= 256) {
    const bool wide = sizeof(T) == 4 ? (mode != SM_FWD_CGQ && mode != SM_FWD_CGQF)
                                     : (mode != SM_INV_DIR && mode != SM_FWD_CGQ &&
                                        mode != SM_FWD_RES);
    if (wide) return strided_v<T, N, str_tb<T, N>(), 1024>(mode, a, nrhs, s);
  }
  return strided_v<T, N, str_tb<T, N>(), NT_STRIDED>(mode, a, nrhs, s);
}

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
template <typename T>
hipError_t launch_zmid(int n, const ZmidArgs<T>& a, int64_t nrows, int nrhs, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: return zmid_n<T, L>(a, nrows, nrhs, s);
    WF_FOR_F32(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_zmid<float>(int, const ZmidArgs<float>&, int64_t, int, hipStream_t);
template hipError_t launch_zmid<double>(int, const ZmidArgs<double>&, int64_t, int, hipStream_t);

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

}  // namespace wf
