// Batched 1D complex FFTs on a tile held in LDS (Stockham autosort, mixed
// radix 2/3/4/8), the building block of every 3D pass.
//
// A tile holds NB pencils of length N.  Two layouts:
//   batch-fast (BF = true):  element (b, i) at lds[i * NB + b]  -- tiles cut
//       across a strided axis, loaded as NB contiguous neighbours per row;
//   axis-fast  (BF = false): element (b, i) at lds[b * N + i]  -- contiguous
//       pencils (the z axis).
// Each stage of radix R with Ns = product of the radices already applied
// reads x[j + r N/R] (r < R) for butterfly j, multiplies by the twiddles
// w^(r k), k = j mod Ns, w = exp(-+2 pi i / (Ns R)), applies the length-R DFT
// and writes the results to (j / Ns) Ns R + k + r Ns.  After the last stage
// the pencil holds its DFT in natural order.  Twiddles come from a table
// tw[m] = exp(-2 pi i m / N) (computed on the host in FP64).
#pragma once

#include "common.h"

namespace wf {

template <int... Rs> struct Radices {
  static constexpr int len = sizeof...(Rs);
  static constexpr int r[len] = {Rs...};
};

// Forward plans; the inverse runs the radices in reverse order so that the
// last forward stage and the first inverse stage touch the same elements.
// Every plan ends with an even radix (the x pass relies on it: the moduli
// |m| a thread holds in that stage pair up, see xlam_rows).
template <int N> struct Plan;
template <> struct Plan<8> : Radices<8> {};
template <> struct Plan<12> : Radices<3, 4> {};
template <> struct Plan<16> : Radices<4, 4> {};
template <> struct Plan<24> : Radices<3, 8> {};
template <> struct Plan<32> : Radices<8, 4> {};
template <> struct Plan<48> : Radices<3, 4, 4> {};
template <> struct Plan<64> : Radices<8, 8> {};
template <> struct Plan<96> : Radices<3, 8, 4> {};
template <> struct Plan<128> : Radices<8, 4, 4> {};
template <> struct Plan<192> : Radices<3, 8, 8> {};
template <> struct Plan<256> : Radices<8, 8, 4> {};
template <> struct Plan<384> : Radices<3, 8, 4, 4> {};
template <> struct Plan<512> : Radices<8, 8, 8> {};
template <> struct Plan<768> : Radices<3, 8, 8, 4> {};
template <> struct Plan<1024> : Radices<8, 8, 4, 4> {};

template <int N> constexpr int last_radix() { return Plan<N>::r[Plan<N>::len - 1]; }

template <int N> constexpr int plan_radix(int dir, int i) {
  return dir < 0 ? Plan<N>::r[i] : Plan<N>::r[Plan<N>::len - 1 - i];
}
template <int N> constexpr int plan_ns(int dir, int i) {
  int p = 1;
  for (int s = 0; s < i; ++s) p *= plan_radix<N>(dir, s);
  return p;
}

// ---- length-R DFTs, DIR = -1 forward (exp(-i...)), +1 inverse --------------
template <int DIR, typename V> __device__ __forceinline__ void dft2(V& a, V& b) {
  V t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename V> __device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
  V a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_i<DIR>(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

template <int DIR, typename V> __device__ __forceinline__ void dft3(V& x0, V& x1, V& x2) {
  using T = decltype(x0.x);
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  V t = cadd(x1, x2);
  V m = {x0.x - T(0.5) * t.x, x0.y - T(0.5) * t.y};
  V u = mul_i<DIR>(csub(x1, x2));
  u = {u.x * h, u.y * h};
  x0 = cadd(x0, t);
  x1 = cadd(m, u);
  x2 = csub(m, u);
}

template <int DIR, typename V> __device__ __forceinline__ void dft8(V* v) {
  using T = decltype(v[0].x);
  const T c = T(0.70710678118654752440084436210485);  // sqrt(2)/2
  V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // o_k *= exp(DIR 2 pi i k / 8)
  o1 = {c * (o1.x - T(DIR) * o1.y), c * (o1.y + T(DIR) * o1.x)};
  o2 = mul_i<DIR>(o2);
  o3 = {c * (-o3.x - T(DIR) * o3.y), c * (-o3.y + T(DIR) * o3.x)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <int R, int DIR, typename V> __device__ __forceinline__ void dft(V* v) {
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 3) dft3<DIR>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<DIR>(v);
  else static_assert(R == 2, "unsupported radix");
}

template <int N, int NB, bool BF> __device__ __forceinline__ int tile_addr(int b, int i) {
  return BF ? i * NB + b : b * N + i;
}

// One in-place Stockham stage over the whole tile.
template <typename T, int N, int R, int NS, int NB, int NT, bool BF, int DIR>
__device__ __forceinline__ void fft_stage(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  constexpr int NBF = NB * (N / R);
  constexpr int PER = (NBF + NT - 1) / NT;
  constexpr int TWS = N / (NS * R);
  V v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * NT;
    if ((NBF % NT == 0) || bf < NBF) {
      const int b = BF ? bf % NB : bf / (N / R);
      const int j = BF ? bf / NB : bf % (N / R);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[tile_addr<N, NB, BF>(b, j + r * (N / R))];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const V w = tw[r * k * TWS];
          v[i][r] = DIR < 0 ? cmul(v[i][r], w) : cmulc(v[i][r], w);
        }
      }
      dft<R, DIR>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * NT;
    if ((NBF % NT == 0) || bf < NBF) {
      const int b = BF ? bf % NB : bf / (N / R);
      const int j = BF ? bf / NB : bf % (N / R);
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[tile_addr<N, NB, BF>(b, base + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, int NB, int NT, bool BF, int DIR, int I = 0,
          int IEND = Plan<N>::len>
__device__ __forceinline__ void fft_tile(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  if constexpr (I < IEND) {
    constexpr int R = plan_radix<N>(DIR, I);
    constexpr int NS = plan_ns<N>(DIR, I);
    fft_stage<T, N, R, NS, NB, NT, BF, DIR>(lds, tw);
    fft_tile<T, N, NB, NT, BF, DIR, I + 1, IEND>(lds, tw);
  }
}

// Copies the twiddle table into LDS (callers synchronise before use).
template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* __restrict__ src) {
  for (int i = threadIdx.x; i < N; i += NT) dst[i] = src[i];
}

// Forward FFT, multiply by a per-element diagonal, inverse FFT, on a
// batch-fast tile.  The last forward stage, the diagonal and the first
// inverse stage run on the same registers: that thread holds outputs
// j + r N/R of the forward transform, exactly the inputs of its inverse
// butterfly.  lamv[i][r] is the diagonal at element bf_i / NB + r N / R of
// the FFT axis (bf_i the thread's i-th butterfly, R the last radix).
template <typename T, int N, int NB, int NT>
__device__ __forceinline__ void fft_tile_diag(cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                              const T (*lamv)[Plan<N>::r[Plan<N>::len - 1]]) {
  using V = cplx<T>;
  constexpr int L = Plan<N>::len;
  constexpr int R = Plan<N>::r[L - 1];
  constexpr int NS = N / R;  // radices already applied before the last stage
  constexpr int NBF = NB * (N / R);
  constexpr int PER = (NBF + NT - 1) / NT;
  fft_tile<T, N, NB, NT, true, -1, 0, L - 1>(lds, tw);
  V v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * NT;
    if ((NBF % NT == 0) || bf < NBF) {
      const int b = bf % NB, j = bf / NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[tile_addr<N, NB, true>(b, j + r * (N / R))];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[r * j]);
      }
      dft<R, -1>(v[i]);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = V{v[i][r].x * lamv[i][r], v[i][r].y * lamv[i][r]};
      dft<R, +1>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * NT;
    if ((NBF % NT == 0) || bf < NBF) {
      const int b = bf % NB, j = bf / NB;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[tile_addr<N, NB, true>(b, j * R + r)] = v[i][r];
    }
  }
  __syncthreads();
  fft_tile<T, N, NB, NT, true, +1, 1, L>(lds, tw);
}

}  // namespace wf
