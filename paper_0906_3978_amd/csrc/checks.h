// Argument checks of the solver options and the server's requests (host only:
// plain C++, no device calls).  Each returns null when the argument is valid,
// else a message, with the status code to return in *code.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/wiener.h"

namespace wf {

// The integer a C caller stored in an enum-typed field: C lets any int
// through, and reading an out-of-range value as the C++ enum type would be
// undefined, so the checks look at the bytes.
template <typename E> inline int32_t raw_enum(const E& e) {
  static_assert(sizeof(E) == sizeof(int32_t), "enums of the ABI are 32-bit");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

// n = 2^a 3^b with b <= 1 and 8 <= n <= 512
inline bool grid_size_ok(int n) {
  if (n < 8 || n > 512) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  return m == 1 || m == 3;
}

inline const char* opts_error(const wf_solve_opts& o, wf_status* code) {
  *code = WF_EINVAL;
  const int32_t prec = raw_enum(o.precision);
  if (prec != WF_FP64 && prec != WF_MIXED) return "unknown precision";
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return "tol must be finite and >= 0";
  if (o.max_iter < 0) return "max_iter must be >= 0";
  if (!(o.inner_tol >= 0.0) || o.inner_tol >= 1.0) return "inner_tol must be in [0, 1)";
  if (o.max_outer < 0 || o.check_every < 0) return "max_outer and check_every must be >= 0";
  if (o.precond != WF_PRECOND_NONE && o.precond != WF_PRECOND_PRIOR) return "unknown precond";
  if (!std::isfinite(o.err_tol)) return "err_tol must be finite";
  *code = WF_OK;
  return nullptr;
}

// A server request: grid, box, scheme and supersampling, options, a mask in
// [0, 1] that is not zero everywhere, a finite positive prior table of
// 3 (n/2)^2 + 1 entries (entry 0 ignored), galaxies inside [0, L) and fewer
// than 2^24 of them.
inline const char* request_error(const wf_request& r, wf_status* code) {
  *code = WF_EINVAL;
  if (!grid_size_ok(r.n)) return "n must be 2^a 3^b (b <= 1) within [8, 512]";
  if (!(r.box_mpc > 0.0) || !std::isfinite(r.box_mpc)) return "bad box";
  if (!r.w || !r.p_by_m2 || (r.n_gal > 0 && !r.xyz) || r.n_gal < 0) return "null request array";
  if (r.n_gal >= (int64_t(1) << 24)) {
    *code = WF_EOVERFLOW;
    return "n_gal must be < 2^24";
  }
  const int32_t scheme = raw_enum(r.scheme);
  if (scheme < WF_NGP || scheme > WF_TSC || (r.supersample != 1 && r.supersample != 2))
    return "bad scheme or supersample";
  if (const char* e = opts_error(r.opts, code)) return e;
  *code = WF_EINVAL;
  const int64_t m = (int64_t)r.n * r.n * r.n;
  const int64_t lamlen = 3 * (int64_t)(r.n / 2) * (r.n / 2) + 1;
  double sw = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    const double v = r.w[i];
    if (!(v >= 0.0 && v <= 1.0)) return "mask values must be in [0, 1]";
    sw += v;
  }
  if (!(sw > 0.0)) return "mask is zero everywhere";
  for (int64_t j = 1; j < lamlen; ++j)
    if (!(r.p_by_m2[j] > 0.0) || !std::isfinite(r.p_by_m2[j])) return "P(k) must be finite and > 0";
  for (int64_t i = 0; i < 3 * r.n_gal; ++i)
    if (!(r.xyz[i] >= 0.0 && r.xyz[i] < r.box_mpc))
      return "galaxy coordinates must satisfy 0 <= x < L";
  *code = WF_OK;
  return nullptr;
}

}  // namespace wf
