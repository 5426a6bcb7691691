// Kernel argument blocks and launchers (host side of kernels.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace wf {

// ---- live timing ------------------------------------------------------------
// A profiler arms a pair of events; the next kernel launch of this thread
// takes them, and the runtime stamps them with that dispatch's own start and
// end (no marker packets enter the queue, so timing costs the work nothing).
struct TimedLaunch {
  hipEvent_t start = nullptr, stop = nullptr;
};
TimedLaunch& timed_launch();

template <typename F, typename... Args>
inline void klaunch(F kernel, const dim3& grid, const dim3& block, uint32_t shm, hipStream_t s,
                    Args... args) {
  TimedLaunch& t = timed_launch();
  if (t.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, t.start, t.stop, 0, args...);
    t.start = t.stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
  }
}

// ---- z-axis passes (contiguous rows, real <-> half spectrum) --------------
enum ZinMode : int { ZIN_REAL = 0, ZIN_CGP = 1, ZIN_I64 = 2 };
enum ZoutMode : int { ZOUT_REAL = 0, ZOUT_CGQ = 1, ZOUT_RES = 2, ZOUT_APPLY = 3 };

template <typename T> struct ZfwdArgs {
  const T* in;              // ZIN_REAL: rows; ZIN_CGP: r
  T* p;                     // ZIN_CGP: search direction, updated in place
  T* x;                     // ZIN_CGP: iterate, receives the pending alpha p
  const long long* gin;     // ZIN_I64: integer rows
  double unit;              // ZIN_I64: value of one integer unit
  cplx<T>* out_main;        // [row][nkz_out]
  cplx<T>* out_nyq;         // [row] (kz = N/2) or null
  int32_t nkz_out;
  int64_t rhs_in, rhs_main, rhs_nyq;  // per-RHS strides in elements
  const cplx<T>* tw;
  CgState* st;              // may be null
  int32_t skip;             // SKIP_* (needs st)
};

template <typename T> struct ZinvArgs {
  const cplx<T>* in_main;   // [row][N/2]
  const cplx<T>* in_nyq;    // [row]
  int64_t rhs_main, rhs_nyq;
  T* out;                   // real rows
  int64_t rhs_out;
  const T* aux;             // CGQ: p; RES: x; APPLY: v
  int64_t rhs_aux;
  const T* w;               // noise diagonal: the mask (times the RHS's nbar) or,
  int64_t rhs_w;            // with w_scaled, per-RHS arrays nbar w g (stride rhs_w)
  int32_t w_scaled;
  const double* bvec;       // RES: b
  int64_t rhs_b;
  double scale;             // REAL: output scale
  double* partials;         // per RHS: gridDim.x doubles
  const cplx<T>* tw;
  CgState* st;
  int32_t skip;             // SKIP_*
};

// z middle pass of the prior-split operator: spectrum -> real rows -> times
// nbar w (nbar from the RHS state) -> spectrum, in place
template <typename T> struct ZmidArgs {
  cplx<T>* spec_main;       // [row][N/2]
  cplx<T>* spec_nyq;        // [row]
  int64_t rhs_main, rhs_nyq;
  const T* w;               // as in ZinvArgs
  int64_t rhs_w;
  int32_t w_scaled;
  const cplx<T>* tw;
  const CgState* st;        // required
  int32_t skip;             // SKIP_*
  double* partials;         // folded FP32 iteration: per RHS and block, the sum of
                            // nbar w u^2 over the block's real field u (else null)
};

// ---- strided passes (y or x axis), tiles of TB neighbouring pencils -------
// The x-pass modes of the prior-split operator (see split_passes) scale by the
// split factor: INV_SCALE multiplies the input by c / (M sqrt(D)) before the
// inverse FFT; FWD_SCALE multiplies the output by c sqrt(D); FWD_CGQ writes
// q = [m != 0] aux + c sqrt(D) v and the block partial of aux.q; FWD_RES (FP64)
// writes r = b - ([m != 0] aux + c sqrt(D) v) and the block partial of r.r.
// D = 2 for 0 < kz < N/2 and 1 on the kz = 0 and kz = N/2 planes: the half
// spectrum stores each conjugate pair once, and carrying sqrt(D) in the vectors
// makes their plain dot products the full-spectrum inner products.
// INV_DIR is INV_SCALE of the CG direction, formed on the way in: `in` is r,
// the pending x += alpha p is applied and p = r + beta p written back (Seg p, x).
// INV_FOLD (FP32 prior-split CG) also applies the pending r -= alpha q (Seg r,
// q) before the direction and writes the block partials of the new r.r and
// of p.p without the monopole.  Its q holds only the noise part of C A C p,
// q' = c sqrt(D) v: FWD_CGQF writes q' and the block partials of q'.q' and of
// p(0) q'(0) (the monopole's term, nonzero in one block), and reads p for the
// monopole only; INV_FOLD applies r -= alpha ([m != 0] p + q').
enum StrMode : int {
  SM_FWD = 0, SM_INV = 1, SM_FWD_LAM_INV = 2, SM_FWD_CROP = 3,
  SM_INV_SCALE = 4, SM_FWD_SCALE = 5, SM_FWD_CGQ = 6, SM_FWD_RES = 7, SM_INV_DIR = 8,
  SM_INV_FOLD = 9, SM_FWD_CGQF = 10
};

template <typename T> struct Seg {
  const cplx<T>* in;
  cplx<T>* out;
  int64_t in_outer, in_axis, in_batch, in_rhs;
  int64_t out_outer, out_axis, out_batch, out_rhs;
  int32_t n_outer, n_btiles, axis_contig, n_out;
  // x pass: the y index of a column is the outer index (1) or the batch
  // index (0); its kz is the batch index (lam_kz < 0) or lam_kz
  int32_t lam_y_outer, lam_kz, pad0, pad1;
  const cplx<T>* aux;       // split CGQ / RES: vector at the output's positions
  const cplx<double>* bvec; // split RES: b at the output's positions
  cplx<T>* p;               // split INV_DIR: direction and iterate at the input's positions
  cplx<T>* x;
  cplx<T>* r;               // split INV_FOLD: residual (written back) and q
  const cplx<T>* q;
};

template <typename T> struct StrArgs {
  Seg<T> s0, s1;
  int32_t nblk0, nblk1;
  const T* lam;             // x pass: Lambda rows (xlam_rows layout)
  const cplx<T>* tw;
  const CgState* st;        // may be null
  int32_t skip;             // SKIP_* (needs st)
  const T* fac;             // split modes: c over (|my|, |mx|, kz), in blocks of 16 kz:
                            // [|my|][kz / 16][|mx|][kz % 16]
  double in_scale;          // SM_INV_SCALE: 1 / M
  double* partials;         // SM_FWD_CGQ / SM_FWD_RES: per RHS, one per block;
                            // SM_INV_FOLD: per RHS, r.r of every block, then p.p;
                            // SM_FWD_CGQF: per RHS, q'.q' of every block, then p(0) q'(0)
  int64_t rhs_lam, rhs_fac; // per-RHS strides of lam and fac (0: shared)
};

int strided_tb(int n, bool fp64);   // batch width of a strided tile
int split_vec_tile(int n);          // tile width of the prior-split vectors' layout
int zpass_nb(int n, bool fp64);     // pencils (row pairs) per z-pass block
int zpass_blocks(int n, int64_t nrows, bool fp64);  // blocks of one z-pass launch
bool fft_length_supported(int n, bool fp64);

template <typename T> hipError_t launch_zfwd(int n, int mode, const ZfwdArgs<T>& a,
                                             int64_t nrows, int nrhs, hipStream_t s);
template <typename T> hipError_t launch_zinv(int n, int mode, const ZinvArgs<T>& a,
                                             int64_t nrows, int nrhs, hipStream_t s);
template <typename T> hipError_t launch_strided(int n, int mode, const StrArgs<T>& a,
                                                int nrhs, hipStream_t s);
template <typename T> hipError_t launch_zmid(int n, const ZmidArgs<T>& a, int64_t nrows, int nrhs,
                                             hipStream_t s);

// Sums the block partials of one reduction (nparts per RHS, fixed order) and
// updates the CG state: FIN_PQ -> alpha (or breakdown), FIN_RR -> iteration
// bookkeeping, beta and stopping, FIN_RES -> outer_rr.  The folded FP32
// prior-split iteration uses FIN_RRF after INV_FOLD (the new r.r: iteration
// bookkeeping and stopping; p.p) and, after FWD_CGQF, launch_finalize_fold_pq.
enum FinKind : int { FIN_PQ = 0, FIN_RR = 1, FIN_RES = 2, FIN_RRF = 4 };
hipError_t launch_finalize(int kind, const double* partials, int nparts, int skip, CgState* st,
                           int nrhs, hipStream_t s);
// Folded iteration, after FWD_CGQF: p.q = p.p + M sum(nbar w u^2) (the noise
// part by Parseval, from the z middle pass's partials: nzb per RHS), q.q =
// p.p + 2 (M sum(nbar w u^2) - p(0) q'(0)) + q'.q' (from FWD_CGQF's: 2 nxb
// per RHS); alpha, and beta from r.r - 2 alpha p.q + alpha^2 q.q with p.q
// standing in for r.q.
hipError_t launch_finalize_fold_pq(const double* part_z, int nzb, const double* part_x, int nxb,
                                   double m_cells, int skip, CgState* st, int nrhs, hipStream_t s);

// ---- vector kernels --------------------------------------------------------
constexpr int VEC_THREADS = 256;
int vec_blocks(int64_t m);
int update_blocks(int64_t m, bool fp64);   // blocks (= partials per RHS) of the update kernel

// x = 0; r = (T) src; rho = r.r; bnorm; starts a CG solve
template <typename T> hipError_t launch_cg_init(T* x, T* r, const double* src, int64_t m,
                                                int64_t rhs_stride, double* partials,
                                                CgState* st, int nrhs, hipStream_t s);
// r -= alpha q; block partials of r.r (then FIN_RR).  x += alpha p is left
// pending for the next z pass (or a fold / flush).
template <typename T> hipError_t launch_cg_update(T* r, const T* q, int64_t m,
                                                  int64_t rhs_stride, double* partials,
                                                  CgState* st, int nrhs, hipStream_t s);
// x += alpha p for the RHS whose state has it pending, then clears it
template <typename T> hipError_t launch_cg_flush(T* x, const T* p, int64_t m, int64_t rhs_stride,
                                                 CgState* st, int nrhs, hipStream_t s);
// mixed precision with reliable updates:
// start: x64 = 0, r64 = b, x32 = 0, r32 = (float) b; bnorm, rho, rmax
hipError_t launch_rel_init(double* x64, double* r64, const double* b, float* x32, float* r32,
                           int64_t m, int64_t rhs_stride, double* partials, CgState* st, int nrhs,
                           hipStream_t s);
// RHS waiting for an update: x64 += x32 (+ the pending alpha p32), x32 = 0,
// and the relative change of the solution into the state (`move`); with `fac`
// (the FP64 prior-split factor table of an n^3 grid, per-RHS stride fac_rs)
// the vectors are half spectra (spec_main complex in the main part) and the
// change is measured on s = C y
hipError_t launch_rel_fold(double* x64, float* x32, const float* p32, int64_t m,
                           int64_t rhs_stride, double* partials, const double* fac, int n,
                           int64_t spec_main, int64_t fac_rs, CgState* st, int nrhs,
                           hipStream_t s);
// RHS waiting for an update (after r64 = b - A64 x64): r32 = (float) r64, rho,
// convergence test on the FP64 residual, resume or stop.  p32 (folded FP32
// iteration only, else null): the formed direction continues with the new r.
hipError_t launch_rel_reset(float* r32, const double* r64, float* p32, int64_t m,
                            int64_t rhs_stride, double* partials, CgState* st, int nrhs,
                            hipStream_t s);

// state of nrhs solves from device-resident nbar values
hipError_t launch_state_init(CgState* st, const double* nbar, double tol, int32_t max_iter,
                             double delta, int32_t max_updates, double err_tol, int nrhs,
                             hipStream_t s);

// a running mixed solve: ask for a reliable update (done, CG_UPDATE)
hipError_t launch_state_request_update(CgState* st, hipStream_t s);
// marks one solve stopped (done, CG_STOPPED)
hipError_t launch_state_stop(CgState* st, hipStream_t s);

hipError_t launch_fill_i64(long long* p, int64_t n, hipStream_t s);
hipError_t launch_fill_c64(double2* p, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s);
hipError_t launch_f64_to_f32(float* out, const double* in, int64_t n, hipStream_t s);
hipError_t launch_f32_to_f64(double* out, const float* in, int64_t n, hipStream_t s);
hipError_t launch_i64_to_f64(double* out, const long long* in, double unit, int64_t n,
                             hipStream_t s);

// ---- deposit / inputs ------------------------------------------------------
hipError_t launch_check_xyz(const double* xyz, int64_t ngal, double box, int* flag, hipStream_t s);
hipError_t launch_deposit(int scheme, const double* xyz, int64_t ngal, double c, int nd,
                          long long* grid, hipStream_t s);
// validates w (finite, 0 <= w <= 1), copies to w64/w32 and writes sum(w) to *sumw
hipError_t launch_mask(const double* w, double* w64, float* w32, int64_t m, int* flag,
                       double* partials, uint32_t* ticket, double* sumw, hipStream_t s);
// lam[j] = (dv / p[j]) * inv_m for j >= 1, lam[0] = 0; flags non-finite or <= 0
hipError_t launch_lambda(const double* p, int64_t len, double dv, double inv_m, double* lam64,
                         int* flag, hipStream_t s);
// Elements of the x-pass Lambda rows of an n^3 grid, and their expansion from
// the table over |m|^2 (FP64 and FP32 copies).
int64_t xlam_elems(int n);
hipError_t launch_xlam_rows(int n, const double* lam, double* rows64, float* rows32,
                            hipStream_t s);
// Prior-split factor c = Lambda^(-1/2) over (|my|, |mx|, kz) in [0, n/2]^3 from
// the |m|^2 table (which carries 1/M), c at |m|^2 = 1 standing in for the
// monopole; blocks of 16 consecutive kz; FP64 and FP32 copies.
int64_t split_fac_elems(int n);
hipError_t launch_split_fac(int n, const double* lam, double m_cells, double* fac64, float* fac32,
                            hipStream_t s);
// onorm = ||v|| per RHS
hipError_t launch_state_norm(const double* v, int64_t m, int64_t rhs_stride, double* partials,
                             CgState* st, int nrhs, hipStream_t s);
// nbar = ngal / sumw; b = w > 0 ? nobs - nbar w : 0
hipError_t launch_data_vector(const double* nobs, const double* w, const double* sumw, double ngal,
                              double* nbar_out, double* b, int64_t m, hipStream_t s);

}  // namespace wf
