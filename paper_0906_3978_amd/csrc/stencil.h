// Fixed-point mass assignment shared by the deposits (def:ngrid, Sec. 3.1.2):
// coordinates u = x N_d / L in units of 2^-FBITS, per-axis integer weights in
// units of 2^-QBITS (NGP: 1).
#pragma once

#include <hip/hip_runtime.h>

namespace wf {

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

}  // namespace wf
