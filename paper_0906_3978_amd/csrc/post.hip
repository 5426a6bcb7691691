// After the solve (Sec. 3.3.2-3.3.3 and Sec. 4): the angle-averaged
// redshift-distortion factor, Fourier-diagonal filters (the deconvolution of
// eq:DEC, Gaussian smoothing), the inverse-weighting comparator and the
// quality measures of Sec. 4.1.
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"
#include "stencil.h"

namespace wf {

// <K D>_mu = int_0^1 (1 + beta mu^2)^2 / (1 + a mu^2) dmu with a = k^2 sigma^2 / 2
// (Kaiser factor times the Lorentzian damping, Sec. 3.3.3).  Dividing the
// numerator by 1 + a mu^2 gives q1 mu^2 + q0 + r / (1 + a mu^2) with
// q1 = beta^2 / a, q0 = 2 beta / a - beta^2 / a^2, r = (1 - beta / a)^2.  For
// small a those terms cancel; there the integrand is expanded in a instead.
__device__ double rsd_average(double a, double beta) {
  if (a < 0.25) {
    double sum = 0.0, an = 1.0;
    for (int k = 0; k < 40; ++k) {
      sum += an * (1.0 / (2 * k + 1) + 2.0 * beta / (2 * k + 3) + beta * beta / (2 * k + 5));
      an *= -a;
    }
    return sum;
  }
  const double q1 = beta * beta / a;
  const double q0 = 2.0 * beta / a - beta * beta / (a * a);
  const double t = 1.0 - beta / a;
  const double sa = sqrt(a);
  return q1 / 3.0 + q0 + t * t * atan(sa) / sa;
}

__global__ void k_rsd_factor(double dk2, double beta, double sigma, double* out, int64_t len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len; j += stride)
    out[j] = rsd_average(0.5 * dk2 * (double)j * sigma * sigma, beta);
}

// Filter table h(|m|^2) times `scale` (the 1/M of the inverse FFT)
__global__ void k_filter_table(int kind, double dk2, double a, double b, double c,
                               const double* table, int64_t len, double scale, double* out,
                               int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len; j += stride) {
    const double k2 = dk2 * (double)j;
    double h;
    if (kind == WF_FILTER_GAUSS) {
      h = exp(-0.5 * k2 * a * a);
    } else if (kind == WF_FILTER_RSD_DECONV) {
      h = 1.0 / (c * sqrt(rsd_average(0.5 * k2 * b * b, a)));
    } else {
      h = table[j];
    }
    if (!isfinite(h)) atomicOr(flag, 1);
    out[j] = h * scale;
  }
}

hipError_t launch_rsd_factor(double dk2, double beta, double sigma, double* out, int64_t len,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rsd_factor, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 1024)),
                     dim3(256), 0, s, dk2, beta, sigma, out, len);
  return hipGetLastError();
}

hipError_t launch_filter_table(int kind, double dk2, double a, double b, double c,
                               const double* table, int64_t len, double scale, double* out,
                               int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_filter_table, dim3((unsigned)std::min<int64_t>((len + 255) / 256, 1024)),
                     dim3(256), 0, s, kind, dk2, a, b, c, table, len, scale, out, flag);
  return hipGetLastError();
}

// out = F^-1 diag(h) F in through the five FP64 sweeps of the operator, the
// fused x pass taking the filter's x-pass rows (1/M folded in) for Lambda.
Status filter_passes(const OperatorData& od, const double* hrows, const double* in,
                     cplx<double>* spec, double* out, hipStream_t s) {
  const Grid& g = od.g;
  ZfwdArgs<double> zf{};
  zf.in = in;
  zf.out_main = spec;
  zf.out_nyq = spec + g.spec_main;
  zf.nkz_out = g.n / 2;
  zf.rhs_in = g.m;
  zf.rhs_main = g.spec_total;
  zf.rhs_nyq = g.spec_total;
  zf.tw = od.tw64.as<double2>();
  WF_HIP(launch_zfwd<double>(g.n, ZIN_REAL, zf, g.nrows, 1, s));
  WF_HIP(launch_strided<double>(g.n, SM_FWD, spectrum_args<double>(od, spec, false), 1, s));
  StrArgs<double> xa = spectrum_args<double>(od, spec, true);
  xa.lam = hrows;
  WF_HIP(launch_strided<double>(g.n, SM_FWD_LAM_INV, xa, 1, s));
  WF_HIP(launch_strided<double>(g.n, SM_INV, spectrum_args<double>(od, spec, false), 1, s));
  ZinvArgs<double> zi{};
  zi.in_main = spec;
  zi.in_nyq = spec + g.spec_main;
  zi.rhs_main = g.spec_total;
  zi.rhs_nyq = g.spec_total;
  zi.out = out;
  zi.rhs_out = g.m;
  zi.scale = 1.0;
  zi.tw = od.tw64.as<double2>();
  WF_HIP(launch_zinv<double>(g.n, ZOUT_REAL, zi, g.nrows, 1, s));
  return {};
}

// ---- moments and comparisons (block partials, summed on the host in block
// order: deterministic) --------------------------------------------------

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;

// sums of 1, v, v^2, v^3, v^4 over the cells (with w > 0 if w is given)
__global__ __launch_bounds__(RED_THREADS) void k_moments(const double* v, const double* w, int64_t m,
                                                         double* partials) {
  __shared__ double red[RED_THREADS / 64];
  double s[5] = {0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < m; i += stride) {
    if (w && !(w[i] > 0.0)) continue;
    const double x = v[i], x2 = x * x;
    s[0] += 1.0;
    s[1] += x;
    s[2] += x2;
    s[3] += x2 * x;
    s[4] += x2 * x2;
  }
  for (int k = 0; k < 5; ++k) {
    const double t = block_sum(s[k], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 5 + k] = t;
  }
}

// Sec. 4.1: sums of t r, t^2, r^2, (r - t)^2, (1 + r) log((1 + r) / (1 + t)) and
// the cell count, over the cells (with w > 0 if w is given); a cell with
// 1 + r <= 0 or 1 + t <= 0 flags the Kullback-Leibler sum as undefined
__global__ __launch_bounds__(RED_THREADS) void k_compare(const double* rec, const double* tru,
                                                         const double* w, int64_t m,
                                                         double* partials, int* flag) {
  __shared__ double red[RED_THREADS / 64];
  double s[6] = {0, 0, 0, 0, 0, 0};
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < m; i += stride) {
    if (w && !(w[i] > 0.0)) continue;
    const double r = rec[i], t = tru[i];
    s[0] += t * r;
    s[1] += t * t;
    s[2] += r * r;
    s[3] += (r - t) * (r - t);
    if (1.0 + r > 0.0 && 1.0 + t > 0.0) s[4] += (1.0 + r) * log((1.0 + r) / (1.0 + t));
    else bad = true;
    s[5] += 1.0;
  }
  if (bad) atomicOr(flag, 1);
  for (int k = 0; k < 6; ++k) {
    const double t = block_sum(s[k], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 6 + k] = t;
  }
}

static int red_blocks(int64_t m) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((m + RED_THREADS - 1) / RED_THREADS, RED_BLOCKS));
}

Status field_sums(const double* v, const double* w, int64_t m, DevBuf& parts, const Allocator& al,
                  double out[5], hipStream_t s) {
  const int nb = red_blocks(m);
  WF_TRY(parts.ensure(al, (size_t)nb * 5 * 8));
  hipLaunchKernelGGL(k_moments, dim3(nb), dim3(RED_THREADS), 0, s, v, w, m, parts.as<double>());
  WF_HIP(hipGetLastError());
  std::vector<double> h((size_t)nb * 5);
  WF_HIP(hipMemcpyAsync(h.data(), parts.p, h.size() * 8, hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 5; ++k) out[k] = 0.0;
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 5; ++k) out[k] += h[(size_t)b * 5 + k];
  return {};
}

// ---- allocation-free moments ---------------------------------------------
// Scratch of field_sums_noalloc: the block partials of k_moments (at most
// RED_BLOCKS x 5 doubles) and the 5 sums.  A file-scope device array: one copy
// per GPU, held until the process ends.  Its host-side name is not a device
// address; host code uses the address hipGetSymbolAddress returns for the
// current device.  Every call on a GPU uses that GPU's copy: calls that
// overlap on one GPU race.  Nothing in it needs clearing: k_moments writes
// every partial it uses and k_sum_parts every sum.
constexpr int NOALLOC_PARTS = RED_BLOCKS * 5;
constexpr int NOALLOC_DOUBLES = NOALLOC_PARTS + 8;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_addr[MAX_DEVICES] = {};   // device address of `scratch` per GPU

// The device address of `scratch` on `device`, which must be current: taken
// once per device and kept.
Status scratch_of(int device, double** out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(WF_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_addr[device]) {
    void* p = nullptr;
    WF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(WF_EDEVICE, "hipGetSymbolAddress returned a null address");
    scratch_addr[device] = static_cast<double*>(p);
  }
  *out = scratch_addr[device];
  return {};
}
}  // namespace

// out[k] = sum over blocks b of parts[b * ncomp + k], in block order (the
// order the host uses in field_sums, so both give the same bits)
__global__ void k_sum_parts(const double* __restrict__ parts, int nb, int ncomp, double* out) {
  if (blockIdx.x == 0 && (int)threadIdx.x < ncomp) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += parts[(int64_t)b * ncomp + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

Status field_sums_noalloc(const double* v, const double* w, int64_t m, int device, double out[5],
                          hipStream_t s) {
  const int nb = red_blocks(m);
  if ((int64_t)nb * 5 > NOALLOC_PARTS)
    return fail(WF_EINVAL, "reduction needs more partials than the static scratch holds");
  double* sc = nullptr;
  WF_TRY(scratch_of(device, &sc));
  hipLaunchKernelGGL(k_moments, dim3(nb), dim3(RED_THREADS), 0, s, v, w, m, sc);
  WF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, sc, nb, 5, sc + NOALLOC_PARTS);
  WF_HIP(hipGetLastError());
  WF_HIP(hipMemcpyAsync(out, sc + NOALLOC_PARTS, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  return {};
}

void moments_from_sums(const double sm[5], double out5[5]) {
  const double n = sm[0];
  double res[5] = {n, NAN, NAN, NAN, NAN};
  if (n > 0) {
    const double mu = sm[1] / n;
    const double e2 = sm[2] / n, e3 = sm[3] / n, e4 = sm[4] / n;
    const double var = e2 - mu * mu;
    const double m3 = e3 - 3 * mu * e2 + 2 * mu * mu * mu;
    const double m4 = e4 - 4 * mu * e3 + 6 * mu * mu * e2 - 3 * mu * mu * mu * mu;
    res[1] = mu;
    res[2] = var;
    if (var > 0) {
      res[3] = m3 / std::pow(var, 1.5);
      res[4] = m4 / (var * var) - 3.0;
    }
  }
  for (int k = 0; k < 5; ++k) out5[k] = res[k];
}

Status compare_sums(const double* rec, const double* tru, const double* w, int64_t m, DevBuf& parts,
                    DevBuf& flag, const Allocator& al, double out[6], bool* kl_ok, hipStream_t s) {
  const int nb = red_blocks(m);
  WF_TRY(parts.ensure(al, (size_t)nb * 6 * 8));
  WF_TRY(flag.ensure(al, sizeof(int)));
  WF_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_compare, dim3(nb), dim3(RED_THREADS), 0, s, rec, tru, w, m,
                     parts.as<double>(), flag.as<int>());
  WF_HIP(hipGetLastError());
  std::vector<double> h((size_t)nb * 6);
  int bad = 0;
  WF_HIP(hipMemcpyAsync(h.data(), parts.p, h.size() * 8, hipMemcpyDeviceToHost, s));
  WF_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  WF_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 6; ++k) out[k] = 0.0;
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 6; ++k) out[k] += h[(size_t)b * 6 + k];
  *kl_ok = bad == 0;
  return {};
}

// ---- inverse weighting (Sec. 4, def:ngrid with the 1/w weights) -----------

// Each galaxy carries 1/w of the target node nearest to it (fixed point on the
// target grid as in the deposit) and is deposited with its stencil on the
// deposit grid in FP64 (atomic sums: the order of the additions is not fixed,
// so the result is reproducible to rounding, not bit for bit).
template <int SCHEME>
__global__ __launch_bounds__(256) void k_deposit_iw(const double* __restrict__ xyz, int64_t ngal,
                                                    double c, int nd, double ct, int n,
                                                    const double* __restrict__ w, double* grid,
                                                    int* flag) {
  constexpr int S = SCHEME + 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngal) return;
  long long first[3], wts[3][3];
  long long node[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double x = xyz[g * 3 + a];
    double u = __dmul_rn(x, c);
    if (u >= (double)nd) u -= (double)nd;
    const long long U = (long long)floor(u * (double)(1LL << FBITS));
    axis_stencil<SCHEME>(U, first[a], wts[a]);
    double ut = __dmul_rn(x, ct);
    if (ut >= (double)n) ut -= (double)n;
    const long long Ut = (long long)floor(ut * (double)(1LL << FBITS));
    node[a] = ((Ut + (1LL << (FBITS - 1))) >> FBITS) % n;
  }
  const double wv = w[(node[0] * n + node[1]) * n + node[2]];
  if (!(wv > 0.0)) {
    atomicOr(flag, 1);
    return;
  }
  const double unit = (SCHEME == 0 ? 1.0 : 1.0 / (double)(1LL << (3 * QBITS))) / wv;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const long long ix = (first[0] + i + nd) % nd;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const long long iy = (first[1] + j + nd) % nd;
      const long long wxy = wts[0][i] * wts[1][j];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const long long iz = (first[2] + k + nd) % nd;
        const long long wt = wxy * wts[2][k];
        if (wt) atomicAdd(grid + ((ix * nd + iy) * nd + iz), (double)wt * unit);
      }
    }
  }
}

hipError_t launch_deposit_iw(int scheme, const double* xyz, int64_t ngal, double c, int nd,
                             double ct, int n, const double* w, double* grid, int* flag,
                             hipStream_t s) {
  if (ngal <= 0) return hipSuccess;
  dim3 gd((unsigned)((ngal + 255) / 256));
  switch (scheme) {
    case 0: hipLaunchKernelGGL(k_deposit_iw<0>, gd, dim3(256), 0, s, xyz, ngal, c, nd, ct, n, w, grid, flag); break;
    case 1: hipLaunchKernelGGL(k_deposit_iw<1>, gd, dim3(256), 0, s, xyz, ngal, c, nd, ct, n, w, grid, flag); break;
    case 2: hipLaunchKernelGGL(k_deposit_iw<2>, gd, dim3(256), 0, s, xyz, ngal, c, nd, ct, n, w, grid, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// delta = n / nbar - 1
__global__ void k_overdensity(double* v, int64_t m, double inv_nbar) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
    v[i] = v[i] * inv_nbar - 1.0;
}

hipError_t launch_overdensity(double* v, int64_t m, double inv_nbar, hipStream_t s) {
  hipLaunchKernelGGL(k_overdensity, dim3((unsigned)std::min<int64_t>((m + 255) / 256, 4096)),
                     dim3(256), 0, s, v, m, inv_nbar);
  return hipGetLastError();
}

}  // namespace wf
