// Internal declarations shared by the HIP sources of libscsf (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>

#include "../../include/scsf.h"

namespace scsf {

// Largest block width the small dense kernels handle (Gram, Cholesky, Jacobi).
constexpr int kMaxK = 256;
constexpr int kMaxDegree = 128;   // largest Chebyshev degree of one filter call
// The FP32 residual-form filter: its correction block left the FP32 range at degree 128 on
// the anisotropic workload (non-finite Ritz values), so mixed precision stops at 64.
constexpr int kMaxDegreeMixed = 64;
// Row chunk processed by one workgroup of the tall-skinny Gram kernel.
constexpr int kGramChunk = 2048;

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side operator descriptor of one problem in a batch.
struct OpDev {
  int32_t kind;
  int32_t N;          // grid side (stencil kinds)
  int64_t n;
  const double *wx, *wy, *v;
  const double *cell;
  const int32_t *row_ptr, *col_idx;
  const double *val;
};

// Which columns of a k-wide block a batched kernel works on, per problem b:
//   ALL            : [0, k)                         (no lock array)
//   ACTIVE         : [lock[b], k)
//   LOCKED         : [0, lock[b])
enum ColMode : int32_t { COLS_ALL = 0, COLS_ACTIVE = 1, COLS_LOCKED = 2 };

__host__ __device__ inline void col_range(int32_t mode, int32_t k, const int32_t *lock, int b,
                                          int32_t &c0, int32_t &cnt) {
  int32_t l = lock ? lock[b] : 0;
  if (mode == COLS_LOCKED) { c0 = 0; cnt = l; }
  else if (mode == COLS_ACTIVE) { c0 = l; cnt = k - l; }
  else { c0 = 0; cnt = k; }
  if (cnt < 0) cnt = 0;
}

// ----------------------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipSuccess or the launch error.

// Y[:, c] = a*(A X[:, c]) + bcoef*X[:, c] + g*Z[:, c] for the columns selected by (mode, k,
// lock), per problem coefficients coef[3*b + {0,1,2}] (device).  Z may be null when g == 0
// for every problem (flag has_z = false).  Blocks of problem b start at base + b*bs.
// Nmax: the largest grid side of the stencil problems in the batch (sizes the LDS staging;
// 0 for CSR).  tile: 1, 2 or 4 columns per thread of the LDS-staged form (autotuned).
// pot: some 5-point problem of the batch may carry a potential (op.v); false selects the form
// without the per-node check and is only valid when no problem ever has one.
// cdeg (nullable, B*k): per-column degrees of the adaptive filter; a column takes part while
// step < its degree raised by at most 2 to mtot's residue mod 3 (mtot = the iteration's degree).
hipError_t spmm_step(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                     const double *X, const double *Z, double *Y, int64_t ld, int64_t bs,
                     int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                     bool has_z, hipStream_t st, const int32_t *mdeg = nullptr,
                     int32_t step = 0, int tile = 4, bool pot = true,
                     const int32_t *cdeg = nullptr, int32_t mtot = 0);

// S consecutive FP64 steps in one launch for the grid stencils (temporal blocking):
// from level i (Xc) and level i-1 (Xp; null when i = 0) to level i+S (Ocur) and i+S-1 (Oprev).
// coef: the S steps' (a, b, g), step t at coef[(t B + b) 3 + {0,1,2}].  Ocur and Oprev must not
// overlap Xc or Xp.  Problems with mdeg[b] <= step0 are skipped (their degree is aligned so
// that no problem ends inside a group).  spmm_fused_supported: the kind has the fused form
// and its LDS arrays fit for grid side Nmax and S steps.
bool spmm_fused_supported(int32_t kind, int32_t Nmax, int S);
hipError_t spmm_fused(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                      const double *Xc, const double *Xp, double *Ocur, double *Oprev,
                      int64_t ld, int64_t bs, int32_t mode, int32_t k, const int32_t *lock,
                      const double *coef, int S, hipStream_t st, const int32_t *mdeg = nullptr,
                      int32_t step0 = 0, int tile = 2, bool pot = true);

// FP32 variant of the step for the mixed-precision filter; with R non-null the step adds the
// per-column source term src[b*k + c] * R[:, c] (R in the same layout as X).
hipError_t spmm_step32(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                       const float *X, const float *Z, float *Y, int64_t ld, int64_t bs,
                       int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                       bool has_z, const float *R, const double *src, hipStream_t st,
                       const int32_t *mdeg = nullptr, int32_t step = 0, int tile = 4,
                       bool pot = true);

// Mixed-precision filter helpers (residual form of the recurrence, see misc.hip):
//  mp_tables : src[(i*B + b)*k + c] = (2 sigma_{i+1}/e) p_i(theta_c) for steps i = 1..m-1 and
//              gain[b*k + c] = p_m(theta_c), from the window written by cheb_coeffs (win).
//  mp_prep   : R32 = fp32(W - theta X), E1 = fp32((sigma_1/e) (W - theta X)) (active columns).
//  mp_final  : Y = X diag(gain) + fp64(Em) (active columns).
hipError_t mp_tables(int B, int32_t k, int32_t m, const double *theta, const double *win,
                     const int32_t *lock, const int32_t *done, double *src, double *gain,
                     const int32_t *mdeg, hipStream_t st);
hipError_t mp_prep(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, const int32_t *lock,
                   const double *X, const double *W, const double *theta, const double *coef,
                   float *R32, float *E1, hipStream_t st);
hipError_t mp_final(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, const int32_t *lock,
                    const double *X, const float *Em, const double *gain, double *Y,
                    hipStream_t st);

// Partial tall-skinny products C_b = A_b^T B_b over row chunks; then reduce.
//   A_b = A + b*bsA + a0*ld, B_b = Bm + b*bsB + b0*ld (column ranges from modes),
//   C_b = C + b*ldc*ldc (ldc x ldc, column-major), entries outside the ranges untouched.
//   symmetric = true: A and B are the same block/range, only upper tiles computed and C is
//   symmetrised.
//   rows (nullable): rows[b] <= n rows of problem b take part (a batch of uneven sizes in
//   blocks of leading dimension ld); null means n rows for every problem.
hipError_t gemm_tn(int B, int64_t n, int64_t ld, const double *A, int64_t bsA, int32_t modeA,
                   const double *Bm, int64_t bsB, int32_t modeB, int32_t k, const int32_t *lock,
                   bool symmetric, double *partial, int64_t partial_stride, double *C, int32_t ldc,
                   const int32_t *gate, int32_t gate_mask, hipStream_t st,
                   const int32_t *rows = nullptr);
int64_t gemm_tn_partial_elems(int64_t n, int32_t ldc);

// Out_b[:, cols(modeO)] = beta*Out + alpha * In_b[:, cols(modeI)] * M_b,
// M_b = M + b*ldm*ldm, (rows = |cols(modeI)|, columns = |cols(modeO)|), column-major ldm.
// In and Out may be the same block when beta == 0 (in-place rotation).
// gate (nullable): only problems with gate[b] & gate_mask run; skip (nullable): problems with
// skip[b] & skip_mask are left untouched (a failed factorisation is never applied).
// rows (nullable): only the first rows[b] rows of problem b are computed and written.
hipError_t gemm_nn(int B, int64_t n, int64_t ld, const double *In, int64_t bsI, int32_t modeI,
                   double *Out, int64_t bsO, int32_t modeO, int32_t k, const int32_t *lock,
                   const double *M, int32_t ldm, double alpha, double beta, const int32_t *gate,
                   int32_t gate_mask, const int32_t *skip, int32_t skip_mask, hipStream_t st,
                   const int32_t *rows = nullptr);

// Per problem b (columns ACTIVE of width ka = k - lock[b]): scaled Cholesky of the Gram
// matrix G_b (ldm x ldm) and the inverse factor M_b = D^-1 R^-1 with D = diag(sqrt(G_jj)),
// R^T R = D^-1 G D^-1.  If a pivot is not positive the factorisation is retried once with the
// CholeskyQR shift s = 11 (n ka + ka (ka+1)) u trace(G) (flag bit 4).  flag[b] |= 1 on
// breakdown, 2 on NaN/Inf.  gate (nullable): only problems with gate[b] & gate_mask run.
// scratch: B * kMaxK * (kMaxK+1) doubles (used when k is too large for LDS).
hipError_t chol_inv(int B, int64_t n, int32_t k, const int32_t *lock, const double *G, double *M,
                    int32_t ldm, int32_t *flag, const int32_t *gate, int32_t gate_mask,
                    double *scratch, hipStream_t st);

// Per problem: symmetric eigendecomposition of the ACTIVE projected matrix G_b (ka x ka) by
// parallel cyclic Jacobi.  Eigenvalues ascending into theta[b*k + lock[b] + j], eigenvectors
// into Z_b (ldm x ldm).  scratch: B * kMaxK * (kMaxK+1) doubles (matrices too large for LDS);
// rec: B * jacobi_record_elems(k) doubles (recorded rotations); ranks: B * ldm ints;
// nsweeps: B ints.  flag bit 8: not converged within the sweep limit.
// stop: the sweeps end once the largest relative off-diagonal entry |g_pq| / sqrt|g_pp g_qq|
// is at most `stop` (checked before the first sweep and after each one).
hipError_t jacobi_eig(int B, int32_t k, const int32_t *lock, double *G, double *Z, int32_t ldm,
                      double *theta, int32_t *flag, double *scratch, double *rec,
                      int32_t *ranks, int32_t *nsweeps, hipStream_t st, double stop = 1e-14);
int64_t jacobi_record_elems(int32_t k);

// The same decomposition without sweeps: Householder tridiagonalisation in LDS, Sturm
// bisection for the eigenvalues (ascending into theta[b*k + lock[b] + j]) and inverse
// iteration for the eigenvectors, back-transformed into Z_b (ldm x ldm, column j = the
// eigenvector of the j-th smallest eigenvalue).  scratch as for jacobi_eig (widths whose packed
// matrix exceeds LDS); work: B * tridiag_work_elems(k) doubles.  flag bit 2: NaN/Inf.
hipError_t tridiag_eig(int B, int32_t k, const int32_t *lock, const double *G, double *Z,
                       int32_t ldm, double *theta, int32_t *flag, double *scratch, double *work,
                       hipStream_t st);
int64_t tridiag_work_elems(int32_t k);

// res[b*k + c] = ||W c - theta c X c|| / ||W c|| for the active columns (over rows[b] rows
// when rows is given).
hipError_t residuals(int B, int64_t n, int64_t ld, const double *X, const double *W,
                     int64_t bs, int32_t k, const int32_t *lock, const double *theta, double *res,
                     hipStream_t st, const int32_t *rows = nullptr);

// Lock the longest converged ascending prefix of the active columns: nconv[b] grows by the
// prefix with res <= tol.  lock[b] (first active column) follows nconv[b], and becomes k
// (done[b] = 1, which makes every ACTIVE-mode kernel skip the problem) once the wanted pairs
// are converged.  mode 0: at least L converged pairs lie at or below the smallest unconverged
// Ritz value theta[nconv[b]] (the L smallest converged pairs are then the wanted ones);
// mode 1: the same in |theta| (squared filter); mode 2 (smallest |theta| from the lower
// end): the q converged pairs at or below theta[nconv[b]] hold L with |theta| <= their
// largest; when no unconverged pair is left first, the problem ends with flag bit 16.
// offv, Lv (nullable, B each): per-slot widths, problem b in columns [offv[b], k) wanting
// Lv[b] pairs (columns below offv[b] are zero placeholders, locked from the start).
hipError_t lock_update(int B, int32_t k, int32_t L, double tol, int32_t *lock, int32_t *nconv,
                       const double *res, const double *theta, int mode, int32_t *done,
                       int32_t *flag, hipStream_t st, const int32_t *offv = nullptr,
                       const int32_t *Lv = nullptr);

// Chebyshev step coefficients for degree m: coef[(s*B + b)*3 + {0,1,2}] for s = 0..m-1 from
// lambda = theta[b*k + offv[b]] (offv null: theta[b*k]), alpha = theta[b*k + k-1] (or win[] when
// given), beta = bounds[b*4+3].
// win (nullable) receives (lambda, c, e) per problem.  hint (nullable): per problem
// (lambda_1, lambda_{L+1}, state); state 1 = apply once if the bounds accept it (-> 2 used,
// 3 rejected).
hipError_t cheb_coeffs(int B, int32_t k, int32_t m, const double *theta, const double *bounds,
                       const int32_t *done, double *coef, double *win, double *hint,
                       hipStream_t st, double *coef2 = nullptr, const int32_t *offv = nullptr);
// Same from explicit (lambda, c, e) per problem: win[b*3 + {0,1,2}].
hipError_t cheb_coeffs_explicit(int B, int32_t m, const double *win, double *coef,
                                hipStream_t st);

// Gershgorin + s-step Lanczos bounds for each problem with need[b] != 0 (need may be null):
// bounds[b*4 + {0,1,2,3}] = (gershgorin, theta_max + beta_s, theta_min, min(g, lanczos)).
// work: B * 3 * nmax doubles.
// square: bounds of A^2 instead (Gershgorin and Lanczos intervals of A, larger end squared).
// key0: the Lanczos start vector of problem b is keyed by key0 + b (a slot, or an operator
// index when all operators of a sequence are bounded up front).
hipError_t bounds(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t steps,
                  uint64_t seed, const int32_t *need, double *work, double *out, hipStream_t st,
                  bool square = false, uint32_t key0 = 0);
// square-mode filter helpers (misc.hip)
hipError_t axpby_active(int B, int64_t nmax, int64_t ld, int64_t bs, int32_t k,
                        const int32_t *lock, const double *X, const double *Z, const double *coef,
                        double *P, const int32_t *rows, hipStream_t st);
hipError_t magnitude_order(int B, int32_t k, const int32_t *lock, double *theta, const double *Z,
                           double *Zout, int32_t ldm, hipStream_t st);

// Fill columns [0, k) of X_b (rows < n) with i.i.d. N(0,1) from Philox4x32-10 keyed by
// (seed, b); rows [n, ld) are zeroed.
hipError_t gaussian_fill(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, double *X,
                         uint64_t seed, hipStream_t st);

// Copy ncols columns (rows < n) between blocks of different leading dimensions; zero_pad also
// zeroes rows [n, ldd) of the destination (internal blocks only, never a caller's buffer).
hipError_t copy_block(int64_t n, int32_t ncols, const double *src, int64_t lds, double *dst,
                      int64_t ldd, bool zero_pad, hipStream_t st);
// X[p, c] /= sqrt(rho[p]) for p < n, c < ncols (plate eigenvectors to M-orthonormal form)
hipError_t scale_rows_rsqrt(int64_t n, int32_t ncols, double *X, int64_t ld, const double *rho,
                            hipStream_t st);

hipError_t fill_int(int32_t *a, int32_t v, int32_t count, hipStream_t st);
// X[p, c] = 0 for p < n, c < ncols
hipError_t zero_columns(int64_t n, int32_t ncols, double *X, int64_t ld, hipStream_t st);
// Per-column degrees of the adaptive filter for the next outer iteration (cdeg: B*k, columns
// [lock[b], k)) and their maximum per problem (mdeg); problems with done[b] are left alone.
hipError_t adaptive_degrees(int B, int32_t k, const int32_t *lock, const int32_t *done,
                            const double *theta, const double *res, const double *bnd,
                            double tol, int32_t mlo, int32_t mhi, int32_t *cdeg, int32_t *mdeg,
                            hipStream_t st);
// Bilinear transfer of ncols nodal fields from the N0 x N0 to the N1 x N1 interior grid of
// the unit square (zero Dirichlet boundary); X and Y must not overlap.
hipError_t interpolate_fields(int32_t N0, int32_t N1, int32_t ncols, const double *X,
                              int64_t ldx, double *Y, int64_t ldy, hipStream_t st);
// dst[:, j] = +-src[:, perm[j]] for j < ncols (rows < n), each column in canonical sign: its
// largest-magnitude entry (lowest row on ties) positive.  src and dst must not overlap.  With
// vals and vout (device, ncols) set, also vout[j] = vals[j].
hipError_t gather_columns_signed(int64_t n, int32_t ncols, const double *src, int64_t lds,
                                 const int32_t *perm, double *dst, int64_t ldd, hipStream_t st,
                                 const double *vals = nullptr, double *vout = nullptr);

// Truncated DFT features and the greedy order.
// sort diagnostics (diag.hip)
constexpr int kMaxDistQ = 32;                   // largest subspace dimension of the distance
hipError_t highfreq_ratio(const double *fields, int32_t n_op, int32_t channels, int32_t p,
                          int32_t p0, double *ratio, hipStream_t st);
hipError_t subspace_distance(int64_t n, int32_t q, const double *X, int64_t ld, int64_t bs,
                             const int32_t *pa, const int32_t *pb, int32_t P, double *out,
                             hipStream_t st);
hipError_t dft_features(const double *fields, int32_t n_op, int32_t channels, int32_t p,
                        int32_t p0, double *feats, hipStream_t st);
hipError_t pair_distances(const double *feats, int32_t n_op, int32_t flen, double *D,
                          hipStream_t st);
hipError_t greedy_order(const double *D, int32_t n_op, int32_t start, int32_t *order,
                        hipStream_t st);

}  // namespace scsf
