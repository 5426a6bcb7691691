// Signal-dependent noise formulation of the Wiener filter (eq:noisecov with
// the count estimators of Sec. 3.4).
//
// With lambda^o the estimate of the expected observed count w lambda per cell
// and g = nbar w / lambda^o on cells with w > 0, the signal-space system of
// eq:WF with N = diag(lambda^o / nbar^2) reads
//   (F^-1 Lambda F + diag(nbar w g)) s = g (n^o - nbar w),
// i.e. the LSQ operator with its noise diagonal replaced by per-RHS arrays;
// lambda^o = nbar w gives back the LSQ system.  Estimators:
//   mean      : lambda^o = N^o_c + 1 (flat prior, Sec. 3.4.1)
//   jackknife : each galaxy kept with probability alpha / w of its node,
//               lambda^o = w (N' + 1) / alpha (eq:selfunc, read with the same
//               flat-prior + 1 so that no observed cell has zero noise)
// N^o_c and N' count galaxies by nearest target node.  The jackknife draws
// are Philox4x32-10 (Salmon et al., SC'11) of counter (galaxy index low and
// high words, sample index, 0) and key (seed low and high words); galaxy g is
// kept in sample j when the first output word u satisfies u < (alpha / w) 2^32,
// compared in FP64 (exact on both sides of the comparison).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "solver.h"
#include "stencil.h"

namespace wf {

namespace {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

// first output word of Philox4x32 with 10 rounds
__device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    const uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  return c0;
}

// counts by nearest target node on nodes with w > 0: all galaxies (THIN
// false, K = 1) or, per sample j < K, the galaxies kept by the thinning
template <bool THIN>
__global__ __launch_bounds__(256) void k_sd_counts(const double* __restrict__ xyz, int64_t ngal,
                                                   double ct, int n, const double* __restrict__ w,
                                                   double alpha, uint32_t key0, uint32_t key1,
                                                   int64_t first, int K, int32_t* counts,
                                                   int* flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngal) return;
  long long node[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double x = xyz[g * 3 + a];
    double ut = __dmul_rn(x, ct);
    if (ut >= (double)n) ut -= (double)n;
    const long long Ut = (long long)floor(ut * (double)(1LL << FBITS));
    node[a] = ((Ut + (1LL << (FBITS - 1))) >> FBITS) % n;
  }
  const int64_t i = (node[0] * n + node[1]) * n + node[2];
  const double wv = w[i];
  if (!(wv > 0.0)) return;
  if constexpr (!THIN) {
    atomicAdd(counts + i, 1);
  } else {
    if (alpha > wv) {
      atomicOr(flag, 1);
      return;
    }
    const double thr = (alpha / wv) * 4294967296.0;
    const int64_t m = (int64_t)n * n * n;
    for (int j = 0; j < K; ++j) {
      const uint64_t smp = (uint64_t)(first + j);
      const uint32_t u = philox_word0((uint32_t)g, (uint32_t)((uint64_t)g >> 32), (uint32_t)smp,
                                      0u, key0, key1);
      if ((double)u < thr) atomicAdd(counts + (int64_t)j * m + i, 1);
    }
  }
}

// per sample j: lambda^o from the counts, g = nbar w / lambda^o, the noise
// diagonal nbar w g (FP64 and FP32) and the data vector g (n^o - nbar w)
__global__ __launch_bounds__(256) void k_sd_system(const int32_t* __restrict__ counts,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ nobs, double nbar,
                                                   int jackknife, double alpha, int K, int64_t m,
                                                   double* d64, float* d32, double* b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const double wv = w[i];
    const double nw = nbar * wv;
    const double res = nobs[i] - nw;
    for (int j = 0; j < K; ++j) {
      const int64_t o = (int64_t)j * m + i;
      double d = 0.0, bv = 0.0;
      if (wv > 0.0) {
        const double c1 = (double)counts[o] + 1.0;
        const double lo = jackknife ? wv * c1 / alpha : c1;
        const double gv = nw / lo;
        d = nw * gv;
        bv = gv * res;
      }
      d64[o] = d;
      d32[o] = (float)d;
      b[o] = bv;
    }
  }
}

// sum[i] += x_0[i] + x_1[i] + ... (samples in order: deterministic)
__global__ __launch_bounds__(256) void k_sum_rows(double* sum, const double* __restrict__ x, int K,
                                                  int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    double acc = sum[i];
    for (int j = 0; j < K; ++j) acc += x[(int64_t)j * m + i];
    sum[i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_scale(double* v, int64_t m, double a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) v[i] *= a;
}

dim3 grid_for(int64_t m) { return dim3((unsigned)std::min<int64_t>((m + 255) / 256, 8192)); }

// clears the noise arrays of the operator when a solve ends, however it ends
struct SdGuard {
  OperatorData& od;
  explicit SdGuard(OperatorData& o) : od(o) { od.sd = true; }
  ~SdGuard() {
    od.sd = false;
    od.dg64.release();
    od.dg32.release();
  }
};

}  // namespace

hipError_t launch_sd_counts(bool thin, const double* xyz, int64_t ngal, double ct, int n,
                            const double* w, double alpha, uint64_t seed, int64_t first, int K,
                            int32_t* counts, int* flag, hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  const dim3 gd((unsigned)((ngal + 255) / 256));
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (thin)
    hipLaunchKernelGGL(k_sd_counts<true>, gd, dim3(256), 0, s, xyz, ngal, ct, n, w, alpha, k0, k1,
                       first, K, counts, flag);
  else
    hipLaunchKernelGGL(k_sd_counts<false>, gd, dim3(256), 0, s, xyz, ngal, ct, n, w, alpha, k0, k1,
                       first, 1, counts, flag);
  return hipGetLastError();
}

Status run_sd(const SdRequest& rq, wf_solve_info* infos) {
  OperatorData& od = *rq.od;
  const Allocator& al = *rq.al;
  const Grid& g = od.g;
  const hipStream_t s = rq.stream;
  const int64_t m = g.m;
  const bool jk = rq.kind == WF_NOISE_SD_JACKKNIFE;
  const int chunk = std::min(rq.nsamples, SD_CHUNK);
  const wf_solve_opts& o = rq.opts;
  SolveWork sw;
  WF_TRY(sw.ensure(al, g, chunk, o.precision == WF_FP64, o.precision == WF_MIXED,
                   o.precond == WF_PRECOND_PRIOR));
  DevBuf counts, sum;
  WF_TRY(counts.ensure(al, (size_t)chunk * m * 4));
  WF_TRY(sum.ensure(al, (size_t)m * 8));
  WF_HIP(launch_fill_f64(sum.as<double>(), m, s));
  SdGuard guard(od);
  WF_TRY(od.dg64.ensure(al, (size_t)chunk * m * 8));
  WF_TRY(od.dg32.ensure(al, (size_t)chunk * m * 4));
  const double ct = (double)g.n / g.box;
  Status worst{};
  for (int j0 = 0; j0 < rq.nsamples; j0 += chunk) {
    const int K = std::min(chunk, rq.nsamples - j0);
    WF_HIP(hipMemsetAsync(counts.p, 0, (size_t)K * m * 4, s));
    WF_HIP(hipMemsetAsync(rq.flag, 0, sizeof(int), s));
    WF_HIP(launch_sd_counts(jk, rq.xyz, rq.n_gal, ct, g.n, od.w64.as<double>(), rq.alpha, rq.seed,
                            rq.first + j0, K, counts.as<int32_t>(), rq.flag, s));
    int bad = 0;
    WF_HIP(hipMemcpyAsync(&bad, rq.flag, sizeof bad, hipMemcpyDeviceToHost, s));
    WF_HIP(hipStreamSynchronize(s));
    if (bad) return fail(WF_EINVAL, "alpha exceeds w at the node of a galaxy");
    hipLaunchKernelGGL(k_sd_system, grid_for(m), dim3(256), 0, s, counts.as<int32_t>(),
                       od.w64.as<double>(), rq.nobs, rq.nbar, jk ? 1 : 0, rq.alpha, K, m,
                       od.dg64.as<double>(), od.dg32.as<float>(), sw.b64.as<double>());
    WF_HIP(hipGetLastError());
    SolveRequest sr;
    sr.od = &od;
    sr.al = &al;
    sr.work = &sw;
    sr.nrhs = K;
    std::vector<double> nbar(K, rq.nbar);
    sr.nbar = nbar.data();
    sr.opts = o;
    sr.stream = s;
    Status r = run_solve(sr, infos + j0);
    if (!(r.code == WF_OK || r.code == WF_ENOTCONV || r.code == WF_EBREAKDOWN)) return r;
    if (severity(r.code) > severity(worst.code)) worst = r;
    hipLaunchKernelGGL(k_sum_rows, grid_for(m), dim3(256), 0, s, sum.as<double>(),
                       sw.x64.as<double>(), K, m);
    WF_HIP(hipGetLastError());
    if (rq.samples_out)
      WF_TRY(download(rq.samples_out + (size_t)j0 * m, sw.x64.p, (size_t)K * m * 8, rq.mem, s));
  }
  hipLaunchKernelGGL(k_scale, grid_for(m), dim3(256), 0, s, sum.as<double>(), m,
                     1.0 / (double)rq.nsamples);
  WF_HIP(hipGetLastError());
  WF_TRY(download(rq.mean_out, sum.p, (size_t)m * 8, rq.mem, s));
  WF_HIP(hipStreamSynchronize(s));
  return worst;
}

}  // namespace wf
