// Host-only logic of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the serving arena (random allocate / release
// sequences checked against an independent model of the occupied ranges),
// and the option and request checks.  Prints "OK" and exits 0 when every
// check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <vector>

#include "arena.h"
#include "checks.h"

static int failures = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                \
    }                                                            \
  } while (0)

static void arena_checks() {
  const size_t size = (size_t)64 << 20;
  std::vector<unsigned char> backing(size);  // host stand-in: only addresses are used
  wf::Arena a;
  a.init(backing.data(), size);
  std::mt19937_64 rng(12345);
  std::map<size_t, size_t> live;  // offset -> bytes (granule rounded)
  size_t in_use = 0, peak = 0;
  for (int step = 0; step < 20000; ++step) {
    const bool alloc = live.empty() || (rng() % 100) < 55;
    if (alloc) {
      size_t want = (size_t)(rng() % (1u << 20)) + 1;
      if (rng() % 10 == 0) want = (size_t)(rng() % 300) + 1;
      void* p = a.get(want);
      const size_t rounded = (want + 255) & ~size_t(255);
      if (!p) {
        // first fit failed: no free range may be large enough
        CHECK(in_use + rounded > size || !live.empty());
        continue;
      }
      const size_t off = (size_t)((unsigned char*)p - backing.data());
      CHECK(off % 256 == 0);
      CHECK(off + rounded <= size);
      // no overlap with any live range
      auto it = live.lower_bound(off);
      if (it != live.end()) CHECK(off + rounded <= it->first);
      if (it != live.begin()) {
        --it;
        CHECK(it->first + it->second <= off);
      }
      live[off] = rounded;
      in_use += rounded;
      peak = std::max(peak, in_use);
      std::fill(backing.begin() + off, backing.begin() + off + std::min<size_t>(rounded, 64),
                (unsigned char)step);
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      a.put(backing.data() + it->first);
      in_use -= it->second;
      live.erase(it);
    }
    CHECK(a.in_use == in_use);
  }
  CHECK(a.peak == peak);
  a.put(nullptr);                      // ignored
  a.put(backing.data() + 3 * 256 + 5);  // not an allocation: ignored
  for (auto& kv : live) a.put(backing.data() + kv.first);
  CHECK(a.in_use == 0);
  // everything returned: the free ranges coalesce into one, and the whole
  // arena can be taken again in one piece
  CHECK(a.free_.size() == 1 && a.free_.begin()->second == size);
  void* all = a.get(size);
  CHECK(all == backing.data());
  CHECK(a.get(1) == nullptr);
  a.put(all);
}

static wf_solve_opts good_opts() {
  wf_solve_opts o{};
  o.precision = WF_MIXED;
  o.tol = 1e-6;
  o.max_iter = 100;
  o.precond = WF_PRECOND_PRIOR;
  return o;
}

static void option_checks() {
  wf_status code;
  CHECK(wf::opts_error(good_opts(), &code) == nullptr && code == WF_OK);
  wf_solve_opts o = good_opts();
  o.tol = NAN;
  CHECK(wf::opts_error(o, &code) && code == WF_EINVAL);
  o = good_opts();
  o.tol = -1.0;
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  o.max_iter = -1;
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  o.inner_tol = 1.0;
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  const int32_t bad = 7;  // what a C caller can store in the enum field
  std::memcpy(&o.precision, &bad, sizeof bad);
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  o.precond = 3;
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  o.err_tol = INFINITY;
  CHECK(wf::opts_error(o, &code));
  o = good_opts();
  o.err_tol = -1.0;  // "off" is allowed
  CHECK(wf::opts_error(o, &code) == nullptr);
  for (int n : {8, 12, 16, 24, 96, 384, 512}) CHECK(wf::grid_size_ok(n));
  for (int n : {0, 4, 10, 18, 36, 72, 576, 1024}) CHECK(!wf::grid_size_ok(n));
}

static void request_checks() {
  const int n = 8;
  std::vector<double> w(n * n * n, 0.5), p(3 * 16 + 1, 100.0), xyz = {1.0, 2.0, 3.0, 4.0, 5.0, 6.0};
  wf_request r{};
  r.n = n;
  r.box_mpc = 10.0;
  r.w = w.data();
  r.p_by_m2 = p.data();
  r.xyz = xyz.data();
  r.n_gal = 2;
  r.scheme = WF_CIC;
  r.supersample = 2;
  r.opts = good_opts();
  wf_status code;
  CHECK(wf::request_error(r, &code) == nullptr && code == WF_OK);
  wf_request b = r;
  b.n = 20;
  CHECK(wf::request_error(b, &code) && code == WF_EINVAL);
  b = r;
  b.box_mpc = 0.0;
  CHECK(wf::request_error(b, &code));
  b = r;
  b.n_gal = int64_t(1) << 24;
  CHECK(wf::request_error(b, &code) && code == WF_EOVERFLOW);
  b = r;
  b.supersample = 3;
  CHECK(wf::request_error(b, &code));
  b = r;
  const int32_t bad_scheme = -1;
  std::memcpy(&b.scheme, &bad_scheme, sizeof bad_scheme);
  CHECK(wf::request_error(b, &code));
  b = r;
  b.xyz = nullptr;
  CHECK(wf::request_error(b, &code));
  b = r;
  b.n_gal = 0;
  b.xyz = nullptr;
  CHECK(wf::request_error(b, &code) == nullptr);
  w[17] = 1.5;
  CHECK(wf::request_error(r, &code) && code == WF_EINVAL);
  w[17] = 0.5;
  std::vector<double> zero(n * n * n, 0.0);
  b = r;
  b.w = zero.data();
  CHECK(wf::request_error(b, &code));
  p[7] = -1.0;
  CHECK(wf::request_error(r, &code));
  p[7] = 100.0;
  p[0] = -5.0;  // entry 0 is ignored
  CHECK(wf::request_error(r, &code) == nullptr);
  xyz[4] = 10.0;  // x == L is outside [0, L)
  CHECK(wf::request_error(r, &code));
  xyz[4] = NAN;
  CHECK(wf::request_error(r, &code));
}

int main() {
  arena_checks();
  option_checks();
  request_checks();
  if (failures) {
    std::printf("%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
