/* Minimal use of the C ABI from C: a periodic 64^3 / 256 Mpc box with a
 * spherical-cap selection, a power-law prior, galaxies drawn uniformly
 * inside the observed region, 2x supersampled CIC deposit, and a
 * mixed-precision prior-split Wiener solve.  Host buffers throughout.
 *
 *   cc -O2 -I include paper_0906_3978_amd/examples/wiener_example.c \
 *      -L paper_0906_3978_amd -lwiener -Wl,-rpath,paper_0906_3978_amd -lm -o wiener_example
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "wiener.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define CHECK(call)                                                              \
  do {                                                                           \
    wf_status st_ = (call);                                                      \
    if (st_ != WF_OK) {                                                          \
      fprintf(stderr, "%s: %s (%s)\n", #call, wf_status_str(st_), ctx ? wf_last_error(ctx) : ""); \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform01(void) { /* xorshift64*, 53-bit mantissa */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1.0p-53;
}

int main(void) {
  const int n = 64;
  const double box = 256.0, h = box / n;
  const int64_t m = (int64_t)n * n * n;
  wf_ctx* ctx = NULL;
  if (wf_abi_version() != WF_ABI_VERSION) {
    fprintf(stderr, "library ABI %d, header %d\n", wf_abi_version(), WF_ABI_VERSION);
    return 1;
  }
  CHECK(wf_ctx_create(&ctx, 0, NULL, NULL, NULL, NULL));
  CHECK(wf_set_grid(ctx, n, box));

  /* selection: a 60-degree cap around +z seen from the box centre, exp(-r/150) */
  double* w = malloc(sizeof(double) * m);
  const double c = 0.5 * box;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        const double dx = i * h - c, dy = j * h - c, dz = k * h - c;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const int in = r == 0.0 || (dz >= cos(M_PI / 3) * r && r <= c);
        w[((int64_t)i * n + j) * n + k] = in ? (r == 0.0 ? 1.0 : exp(-r / 150.0)) : 0.0;
      }
  CHECK(wf_set_mask(ctx, w, WF_HOST));

  /* prior: P(k) = A k^-1.5 exp(-(k/0.5)^2) on the |m|^2 lattice (j = 0 unused) */
  const int64_t len = 3 * (int64_t)(n / 2) * (n / 2) + 1;
  double* p = malloc(sizeof(double) * len);
  p[0] = 1.0;
  for (int64_t jj = 1; jj < len; ++jj) {
    const double k = 2.0 * M_PI / box * sqrt((double)jj);
    p[jj] = 2.0e3 * pow(k, -1.5) * exp(-(k / 0.5) * (k / 0.5));
  }
  CHECK(wf_set_power(ctx, p, len, WF_HOST));

  /* galaxies: uniform positions, kept with probability w at their nearest node */
  const int64_t want = 200000;
  double* xyz = malloc(sizeof(double) * 3 * want);
  int64_t ng = 0;
  while (ng < want) {
    double x[3];
    int node[3];
    for (int a = 0; a < 3; ++a) {
      x[a] = uniform01() * box;
      node[a] = ((int)floor(x[a] / h + 0.5)) % n;
    }
    if (uniform01() < w[((int64_t)node[0] * n + node[1]) * n + node[2]]) {
      for (int a = 0; a < 3; ++a) xyz[3 * ng + a] = x[a];
      ++ng;
    }
  }
  CHECK(wf_set_galaxies(ctx, xyz, ng, WF_HOST));
  CHECK(wf_deposit(ctx, WF_CIC, 2));

  wf_solve_opts o = {0};
  o.precision = WF_MIXED;
  o.tol = 1e-7;
  o.max_iter = 100000;
  o.precond = WF_PRECOND_PRIOR;
  double* s = malloc(sizeof(double) * m);
  wf_solve_info info;
  CHECK(wf_solve(ctx, &o, s, WF_HOST, &info));
  double mom[5];
  CHECK(wf_field_moments(ctx, s, 1, mom, WF_HOST));
  printf("n=%d galaxies=%lld nbar=%.4g: %d iterations, %d FP64 residuals, "
         "||b - A s||/||b|| = %.2e, %.1f ms; observed cells %.0f, mean %.3g, variance %.3g\n",
         n, (long long)ng, info.nbar, info.iters_total, info.outer_steps, info.rel_res_true,
         info.time_ms, mom[0], mom[1], mom[2]);
  CHECK(wf_ctx_destroy(ctx));
  free(w);
  free(p);
  free(xyz);
  free(s);
  return 0;
}
