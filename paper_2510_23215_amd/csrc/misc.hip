// Per-iteration bookkeeping kernels: residual norms and locking (Algorithm 3, lock step),
// Chebyshev window coefficients (Algorithm 1 / Section 2.2), the spectral upper bound
// (Gershgorin and Lanczos), the seeded Gaussian start block, block copies and the output
// sign convention.
#include "stencil.h"

namespace scsf {

__device__ inline double block_sum(double v, double *sh) {
  // sum over the block (blockDim.x a multiple of 64, <= 1024); result valid in all threads
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += sh[w];
  return t;
}

__device__ inline double block_max(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = sh[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, sh[w]);
  return t;
}

// grid (k, 1, B): one workgroup per (active column, problem)
__global__ void __launch_bounds__(256) residual_kernel(
    int64_t n, int64_t ld, const double *__restrict__ X, const double *__restrict__ W, int64_t bs,
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ theta,
    double *__restrict__ res, const int32_t *__restrict__ rows) {
  __shared__ double sh[16];
  const int b = blockIdx.z;
  if (rows) n = rows[b];
  const int32_t l = lock ? lock[b] : 0;
  const int c = l + blockIdx.x;
  if (c >= k) return;
  const double th = theta[(int64_t)b * k + c];
  const double *x = X + (int64_t)b * bs + (int64_t)c * ld;
  const double *w = W + (int64_t)b * bs + (int64_t)c * ld;
  double rr = 0.0, ww = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
    const double wv = w[p], d = wv - th * x[p];
    rr += d * d;
    ww += wv * wv;
  }
  rr = block_sum(rr, sh);
  ww = block_sum(ww, sh);
  if (threadIdx.x == 0) res[(int64_t)b * k + c] = (ww > 0.0) ? sqrt(rr / ww) : sqrt(rr);
}

hipError_t residuals(int B, int64_t n, int64_t ld, const double *X, const double *W,
                     int64_t bs, int32_t k, const int32_t *lock, const double *theta, double *res,
                     hipStream_t st, const int32_t *rows) {
  if (B <= 0) return hipSuccess;
  residual_kernel<<<dim3(k, 1, B), 256, 0, st>>>(n, ld, X, W, bs, k, lock, theta, res, rows);
  return hipGetLastError();
}

// nconv[b]: locked pairs; lock[b]: first active column (= k once the problem is done).
// Per-slot widths (offv, Lv non-null): problem b owns columns [offv[b], k) and wants Lv[b]
// pairs; its columns below offv[b] are zero placeholders, locked from the start, and every
// count below starts at offv[b].
// mode 0: the L algebraically smallest; 1: the L smallest |theta| with the squared filter (the
// active range is ordered by |theta|); 2: the L smallest |theta| from the lower end of the
// spectrum (ascending active range).  Flag bit 16: mode 2 ran out of unconverged pairs before
// its certificate held.
__global__ void lock_kernel(int B, int32_t k, int32_t L, double tol, int32_t *__restrict__ lock,
                            int32_t *__restrict__ nconv, const double *__restrict__ res,
                            const double *__restrict__ theta, int mode,
                            int32_t *__restrict__ done, int32_t *__restrict__ flag,
                            const int32_t *__restrict__ offv, const int32_t *__restrict__ Lv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || done[b]) return;
  const int o = offv ? offv[b] : 0;
  if (Lv) L = Lv[b];
  const int32_t j0 = nconv[b];
  int j = j0;
  while (j < k && res[(int64_t)b * k + j] <= tol) ++j;
  nconv[b] = j;
  // The converged pairs at or below the smallest unconverged Ritz value theta_j (the active
  // range [j0, k) is ordered, so theta_j is its smallest unconverged value) are the lowest
  // ones of the spectrum: a converged pair locked earlier above theta_j means a wanted pair
  // entered the block late, and the solve goes on until it has converged.
  const double *th = theta + (int64_t)b * k;
  const bool absval = mode == 1;
  const double tu = (j < k) ? (absval ? fabs(th[j]) : th[j]) : INFINITY;
  bool fin;
  if (mode != 2) {
    int below = j - j0;
    for (int c = o; c < j0; ++c) below += ((absval ? fabs(th[c]) : th[c]) <= tu) ? 1 : 0;
    fin = j - o >= L && below >= L;
  } else {
    // smallest magnitude from the lower end: the q lowest converged values must hold L with
    // |theta| <= their largest, theta_q (every other eigenvalue is >= theta_q)
    double top = -INFINITY;
    int q = 0;
    for (int c = o; c < j; ++c)
      if (th[c] <= tu) { ++q; top = fmax(top, th[c]); }
    int cnt = 0;
    for (int c = o; c < j; ++c)
      if (th[c] <= tu && fabs(th[c]) <= top) ++cnt;
    fin = q >= L && cnt >= L;
    // no certificate can come (not certified, flag bit 16): no pair left to converge, or fewer
    // than L of the block's k values with |theta| <= the largest of them (a certified state
    // has at least L such values, and the Ritz values of a converging block only drift down)
    if (!fin) {
      double big = -INFINITY;
      for (int c = o; c < k; ++c) big = fmax(big, th[c]);
      int within = 0;
      for (int c = o; c < k; ++c) within += (fabs(th[c]) <= big) ? 1 : 0;
      if (j >= k || within < L) {
        fin = true;
        flag[b] |= 16;
      }
    }
  }
  if (fin) { done[b] = 1; lock[b] = k; }
  else lock[b] = j;
}

hipError_t lock_update(int B, int32_t k, int32_t L, double tol, int32_t *lock, int32_t *nconv,
                       const double *res, const double *theta, int mode, int32_t *done,
                       int32_t *flag, hipStream_t st, const int32_t *offv, const int32_t *Lv) {
  if (B <= 0) return hipSuccess;
  lock_kernel<<<(B + 63) / 64, 64, 0, st>>>(B, k, L, tol, lock, nconv, res, theta, mode, done,
                                            flag, offv, Lv);
  return hipGetLastError();
}

// Scaled recurrence of Algorithm 1: sigma_1 = e/(lambda-c), sigma_{i+1} = 1/(2/sigma_1 - sigma_i);
// step 0: Y1 = (sigma_1/e)(A - cI) Y0; step i: Y_{i+1} = (2 sigma_{i+1}/e)(A - cI) Y_i
//                                                  - sigma_i sigma_{i+1} Y_{i-1}.
__device__ inline void write_coeffs(int B, int b, int32_t m, double lam, double c, double e,
                                    double *coef) {
  const double s1 = e / (lam - c);
  coef[(0 * (int64_t)B + b) * 3 + 0] = s1 / e;
  coef[(0 * (int64_t)B + b) * 3 + 1] = -s1 * c / e;
  coef[(0 * (int64_t)B + b) * 3 + 2] = 0.0;
  double s = s1;
  for (int i = 1; i < m; ++i) {
    const double sn = 1.0 / (2.0 / s1 - s);
    coef[((int64_t)i * B + b) * 3 + 0] = 2.0 * sn / e;
    coef[((int64_t)i * B + b) * 3 + 1] = -2.0 * sn * c / e;
    coef[((int64_t)i * B + b) * 3 + 2] = -s * sn;
    s = sn;
  }
}

// Window of Section 2.2 with the reading: lambda = smallest Ritz value, alpha = largest Ritz
// value of the block, beta = upper bound of the spectrum; c = (alpha+beta)/2, e = (beta-alpha)/2.
// A pending hint (hint[b*3+2] == 1: predicted lambda_1, lambda_{L+1}) replaces lambda and alpha
// once, if the Lanczos bounds accept it: lambda_1 <= theta_min(T_s) (a Ritz value bounds
// lambda_1 from above) and lambda_1 < lambda_{L+1} < beta.  The hint state becomes 2 (used)
// or 3 (rejected).
//
// Square mode (smallest |lambda|): the filter polynomial is in A^2, whose Ritz values are
// theta^2; with the pairs ordered by |theta|, lambda = theta_0^2 and alpha = theta_{k-1}^2,
// and coef2 receives (a_s, 0, 1) for the second operator application of each step.
__global__ void cheb_kernel(int B, int32_t k, int32_t m, const double *__restrict__ theta,
                            const double *__restrict__ bnd, const int32_t *__restrict__ done,
                            double *__restrict__ coef, double *__restrict__ win,
                            double *__restrict__ hint, double *__restrict__ coef2,
                            const int32_t *__restrict__ offv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || (done && done[b])) return;
  double lam = theta[(int64_t)b * k + (offv ? offv[b] : 0)];   // the problem's first column
  double alpha = theta[(int64_t)b * k + k - 1];
  if (coef2) {
    lam *= lam;
    alpha *= alpha;
  }
  double beta = bnd[b * 4 + 3];
  if (hint && hint[b * 3 + 2] == 1.0) {
    const double l1 = hint[b * 3 + 0], lk = hint[b * 3 + 1];
    const bool ok = isfinite(l1) && isfinite(lk) && l1 <= bnd[b * 4 + 2] && l1 < lk && lk < beta;
    if (ok) { lam = l1; alpha = lk; }
    hint[b * 3 + 2] = ok ? 2.0 : 3.0;
  }
  const double span = fmax(fabs(alpha), fabs(lam));
  if (!(beta > alpha + 1e-12 * span)) beta = alpha + fmax(1e-3 * span, 1e-300);
  const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
  double l = lam;
  if (!(l < c - 1e-12 * e)) l = c - e;       // lambda must lie below the damped interval
  if (win) { win[b * 3 + 0] = l; win[b * 3 + 1] = c; win[b * 3 + 2] = e; }
  write_coeffs(B, b, m, l, c, e, coef);
  if (coef2)
    for (int s = 0; s < m; ++s) {
      const int64_t o = ((int64_t)s * B + b) * 3;
      coef2[o + 0] = coef[o + 0];
      coef2[o + 1] = 0.0;
      coef2[o + 2] = 1.0;
    }
}

hipError_t cheb_coeffs(int B, int32_t k, int32_t m, const double *theta, const double *bounds,
                       const int32_t *done, double *coef, double *win, double *hint,
                       hipStream_t st, double *coef2, const int32_t *offv) {
  if (B <= 0) return hipSuccess;
  cheb_kernel<<<(B + 63) / 64, 64, 0, st>>>(B, k, m, theta, bounds, done, coef, win, hint,
                                            coef2, offv);
  return hipGetLastError();
}

__global__ void cheb_explicit_kernel(int B, int32_t m, const double *__restrict__ win,
                                     double *__restrict__ coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  write_coeffs(B, b, m, win[b * 3 + 0], win[b * 3 + 1], win[b * 3 + 2], coef);
}

hipError_t cheb_coeffs_explicit(int B, int32_t m, const double *win, double *coef,
                                hipStream_t st) {
  if (B <= 0) return hipSuccess;
  cheb_explicit_kernel<<<(B + 63) / 64, 64, 0, st>>>(B, m, win, coef);
  return hipGetLastError();
}

// ---------------------------------------------------------------- spectral upper bound
// Lanczos bound of Zhou & Li (2011): theta_max(T_s) + beta_s, with Gershgorin's max row sum.
__device__ inline int sturm_count(const double *a, const double *bb, int s, double x) {
  // number of eigenvalues of the s x s tridiagonal (a, bb) below x
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < s; ++i) {
    const double off = (i > 0) ? bb[i - 1] * bb[i - 1] : 0.0;
    d = a[i] - x - ((i > 0) ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

template <int KIND>
__global__ void __launch_bounds__(1024) bounds_kernel(
    const OpDev *__restrict__ ops, int32_t steps, uint64_t seed, const int32_t *__restrict__ need,
    double *__restrict__ work, int64_t nmax, double *__restrict__ out, int square, uint32_t key0) {
  __shared__ double sh[16];
  __shared__ double al[128], be[128], thx[2];
  __shared__ int s_eff;
  const int b = blockIdx.x;
  if (need && !need[b]) return;
  const OpDev op = ops[b];
  const int64_t n = op.n;
  double *v0 = work + (int64_t)b * 3 * nmax, *v1 = v0 + nmax, *w = v1 + nmax;
  const int tid = threadIdx.x, NT = blockDim.x;
  double nrm = 0.0;
  for (int64_t p = tid; p < n; p += NT) {
    const double2 g = gauss2(seed, (uint64_t)p, key0 + (uint32_t)b, 0x4C414E43u);
    v1[p] = g.x;
    v0[p] = 0.0;
    nrm += g.x * g.x;
  }
  nrm = sqrt(block_sum(nrm, sh));
  for (int64_t p = tid; p < n; p += NT) v1[p] /= nrm;
  if (tid == 0) s_eff = steps;
  double bold = 0.0, gmax = -INFINITY, gmin = INFINITY;
  for (int j = 0; j < steps; ++j) {
    __syncthreads();
    double dot = 0.0;
    for (int64_t p = tid; p < n; p += NT) {
      double g, gl;
      const double r = op_row<KIND>(op, p, v1, j == 0 ? &g : nullptr, j == 0 ? &gl : nullptr) -
                       bold * v0[p];
      if (j == 0) { gmax = fmax(gmax, g); gmin = fmin(gmin, gl); }
      w[p] = r;
      dot += r * v1[p];
    }
    const double a = block_sum(dot, sh);
    double ss = 0.0;
    for (int64_t p = tid; p < n; p += NT) {
      const double r = w[p] - a * v1[p];
      w[p] = r;
      ss += r * r;
    }
    const double bt = sqrt(block_sum(ss, sh));
    if (tid == 0) { al[j] = a; be[j] = bt; }
    if (bt == 0.0) { if (tid == 0) s_eff = j + 1; break; }
    for (int64_t p = tid; p < n; p += NT) { v0[p] = v1[p]; v1[p] = w[p] / bt; }
    bold = bt;
  }
  gmax = block_max(gmax, sh);
  __syncthreads();
  gmin = -block_max(-gmin, sh);
  __syncthreads();
  if (tid < 2) {
    const int s = s_eff;
    // Gershgorin interval of T for the bisection brackets
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < s; ++i) {
      const double r = ((i > 0) ? fabs(be[i - 1]) : 0.0) + ((i < s - 1) ? fabs(be[i]) : 0.0);
      lo = fmin(lo, al[i] - r);
      hi = fmax(hi, al[i] + r);
    }
    const int target = (tid == 0) ? 1 : s;      // smallest / largest eigenvalue of T
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
      const double mid = 0.5 * (lo + hi);
      if (sturm_count(al, be, s, mid) >= target) hi = mid; else lo = mid;
    }
    thx[tid] = 0.5 * (lo + hi);
  }
  __syncthreads();
  if (tid == 0) {
    const double tmin = thx[0], tmax = thx[1], bs = fabs(be[s_eff - 1]);
    out[b * 4 + 2] = tmin;
    if (!square) {
      const double lz = tmax + bs;
      out[b * 4 + 0] = gmax;
      out[b * 4 + 1] = lz;
      out[b * 4 + 3] = fmin(gmax, lz);
    } else {
      // bounds of A^2: the larger end of A's Gershgorin interval and of the Lanczos interval
      // [theta_min - beta_s, theta_max + beta_s], squared
      const double g2 = fmax(fabs(gmax), fabs(gmin)), l2 = fmax(fabs(tmin - bs), fabs(tmax + bs));
      out[b * 4 + 0] = g2 * g2;
      out[b * 4 + 1] = l2 * l2;
      out[b * 4 + 3] = fmin(g2 * g2, l2 * l2);
    }
  }
}

hipError_t bounds(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t steps,
                  uint64_t seed, const int32_t *need, double *work, double *out, hipStream_t st,
                  bool square, uint32_t key0) {
  if (B <= 0) return hipSuccess;
  if (steps < 1 || steps > 128) return hipErrorInvalidValue;
  if (kind == SCSF_STENCIL5)
    bounds_kernel<SCSF_STENCIL5><<<B, 1024, 0, st>>>(ops, steps, seed, need, work, nmax, out,
                                                 square ? 1 : 0, key0);
  else if (kind == SCSF_STENCIL9)
    bounds_kernel<SCSF_STENCIL9><<<B, 1024, 0, st>>>(ops, steps, seed, need, work, nmax, out,
                                                 square ? 1 : 0, key0);
  else if (kind == SCSF_PLATE)
    bounds_kernel<SCSF_PLATE><<<B, 1024, 0, st>>>(ops, steps, seed, need, work, nmax, out,
                                                 square ? 1 : 0, key0);
  else
    bounds_kernel<SCSF_CSR><<<B, 1024, 0, st>>>(ops, steps, seed, need, work, nmax, out,
                                                 square ? 1 : 0, key0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- start block, copies, signs
__global__ void gauss_kernel(int64_t n, int64_t ld, int64_t bs, int32_t k, double *__restrict__ X,
                             uint64_t seed) {
  const int b = blockIdx.z, c = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ld || c >= k) return;
  double v = 0.0;
  if (p < n) {
    const uint64_t e = (uint64_t)c * n + p;
    const double2 g = gauss2(seed, e >> 1, (uint32_t)b, 0x58424C4Bu);
    v = (e & 1) ? g.y : g.x;
  }
  X[(int64_t)b * bs + (int64_t)c * ld + p] = v;
}

hipError_t gaussian_fill(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, double *X,
                         uint64_t seed, hipStream_t st) {
  if (B <= 0 || k <= 0) return hipSuccess;
  gauss_kernel<<<dim3((unsigned)ceil_div(ld, 256), k, B), 256, 0, st>>>(n, ld, bs, k, X, seed);
  return hipGetLastError();
}

__global__ void copy_kernel(int64_t n, const double *__restrict__ src, int64_t lds,
                            double *__restrict__ dst, int64_t ldd, int zero_pad) {
  const int c = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[(int64_t)c * ldd + p] = src[(int64_t)c * lds + p];
  else if (zero_pad && p < ldd) dst[(int64_t)c * ldd + p] = 0.0;
}

hipError_t copy_block(int64_t n, int32_t ncols, const double *src, int64_t lds, double *dst,
                      int64_t ldd, bool zero_pad, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return hipSuccess;
  const int64_t rows = zero_pad ? ldd : n;
  copy_kernel<<<dim3((unsigned)ceil_div(rows, 256), ncols), 256, 0, st>>>(n, src, lds, dst, ldd,
                                                                          zero_pad ? 1 : 0);
  return hipGetLastError();
}

__global__ void scale_rows_kernel(int64_t n, double *__restrict__ X, int64_t ld,
                                  const double *__restrict__ rho) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) X[(int64_t)blockIdx.y * ld + p] /= sqrt(rho[p]);
}

hipError_t scale_rows_rsqrt(int64_t n, int32_t ncols, double *X, int64_t ld, const double *rho,
                            hipStream_t st) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  scale_rows_kernel<<<dim3((unsigned)ceil_div(n, 256), ncols), 256, 0, st>>>(n, X, ld, rho);
  return hipGetLastError();
}

}  // namespace scsf

namespace scsf {

__global__ void fill_int_kernel(int32_t *__restrict__ a, int32_t v, int32_t count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = v;
}

hipError_t fill_int(int32_t *a, int32_t v, int32_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  fill_int_kernel<<<(count + 255) / 256, 256, 0, st>>>(a, v, count);
  return hipGetLastError();
}

__global__ void zero_cols_kernel(int64_t n, double *__restrict__ X, int64_t ld) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) X[(int64_t)blockIdx.y * ld + p] = 0.0;
}

hipError_t zero_columns(int64_t n, int32_t ncols, double *X, int64_t ld, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  zero_cols_kernel<<<dim3((unsigned)ceil_div(n, 256), (unsigned)ncols), 256, 0, st>>>(n, X, ld);
  return hipGetLastError();
}

// dst[:, j] = s_j src[:, perm[j]] for j < ncols (rows < n): the gathered columns in canonical
// sign, s_j = -1 when the source column's entry of largest magnitude (lowest row on ties) is
// negative, else 1.  One workgroup of 1024 threads per column.  Each thread scans its rows in
// increasing order with four loads in flight (a strict comparison keeps the lowest row of a
// tie), the workgroup reduces (magnitude, row) pairs, and the second pass over the column
// (from L2) writes it with the sign applied.  With vals and vout set, workgroup j also writes
// vout[j] = vals[j] (the column's eigenvalue).
constexpr int kSignThreads = 1024;
__global__ void __launch_bounds__(kSignThreads) gather_sign_kernel(
    int64_t n, const double *__restrict__ src, int64_t lds, const int32_t *__restrict__ perm,
    double *__restrict__ dst, int64_t ldd, const double *__restrict__ vals,
    double *__restrict__ vout) {
  constexpr int U = 4, NWAVE = kSignThreads / 64;
  __shared__ double sv[NWAVE];
  __shared__ int64_t si[NWAVE];
  __shared__ int flip_s;
  const int j = blockIdx.x, tid = threadIdx.x;
  if (vout && tid == 0) vout[j] = vals[j];
  const double *x = src + (int64_t)perm[j] * lds;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t p0 = tid; p0 < n; p0 += (int64_t)kSignThreads * U) {
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = p0 + (int64_t)u * kSignThreads;
      a[u] = p < n ? fabs(x[p]) : -1.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (a[u] > best) {
        best = a[u];
        bi = p0 + (int64_t)u * kSignThreads;
      }
  }
  // (larger magnitude, then lower row) wins
  auto take = [&](double ob, int64_t oi) {
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  };
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    take(ob, oi);
  }
  if ((tid & 63) == 0) {
    sv[tid >> 6] = best;
    si[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NWAVE; ++w) take(sv[w], si[w]);
    flip_s = x[bi] < 0.0 ? 1 : 0;
  }
  __syncthreads();
  const bool flip = flip_s != 0;
  double *y = dst + (int64_t)j * ldd;
  for (int64_t p = tid; p < n; p += kSignThreads) y[p] = flip ? -x[p] : x[p];
}

hipError_t gather_columns_signed(int64_t n, int32_t ncols, const double *src, int64_t lds,
                                 const int32_t *perm, double *dst, int64_t ldd, hipStream_t st,
                                 const double *vals, double *vout) {
  if (ncols <= 0 || n <= 0) return hipSuccess;
  gather_sign_kernel<<<(unsigned)ncols, kSignThreads, 0, st>>>(n, src, lds, perm, dst, ldd, vals,
                                                               vout);
  return hipGetLastError();
}

}  // namespace scsf

// ------------------------------------------------------------------ mixed-precision filter
// Residual form of the scaled recurrence.  With p_i the scaled Chebyshev polynomials of
// Algorithm 1 and, for one column, x its Ritz vector, theta its Ritz value and r = A x - theta x,
// the difference e_i = p_i(A) x - p_i(theta) x obeys
//   e_0 = 0,  e_1 = (sigma_1/e) r,
//   e_{i+1} = (2 sigma_{i+1}/e)(A - cI) e_i - sigma_i sigma_{i+1} e_{i-1} + (2 sigma_{i+1}/e) p_i(theta) r,
// (p_{i+1}(A) - p_{i+1}(theta) expanded with p_i(A) x = e_i + p_i(theta) x), so that
// p_m(A) x = p_m(theta) x + e_m exactly.  The e recurrence runs in FP32: its rounding error is
// relative to ||e|| ~ ||r||, not to ||p_m(A) x||, so the iteration keeps converging in FP64.
namespace scsf {

__global__ void mp_tables_kernel(int B, int32_t k, int32_t m, const double *__restrict__ theta,
                                 const double *__restrict__ win, const int32_t *__restrict__ lock,
                                 const int32_t *__restrict__ done, double *__restrict__ src,
                                 double *__restrict__ gain, const int32_t *__restrict__ mdeg) {
  const int b = blockIdx.x;
  if (done && done[b]) return;
  if (mdeg) m = mdeg[b];
  const int32_t l = lock ? lock[b] : 0;
  const double c = win[b * 3 + 1], e = win[b * 3 + 2];
  const double s1 = e / (win[b * 3 + 0] - c);
  for (int col = l + threadIdx.x; col < k; col += blockDim.x) {
    const double t = (theta[(int64_t)b * k + col] - c) / e;
    double pm1 = 1.0, p = s1 * t, s = s1;
    for (int i = 1; i < m; ++i) {
      const double sn = 1.0 / (2.0 / s1 - s);
      src[((int64_t)i * B + b) * k + col] = 2.0 * sn / e * p;
      const double pn = 2.0 * sn * t * p - s * sn * pm1;
      pm1 = p;
      p = pn;
      s = sn;
    }
    gain[(int64_t)b * k + col] = p;
  }
}

hipError_t mp_tables(int B, int32_t k, int32_t m, const double *theta, const double *win,
                     const int32_t *lock, const int32_t *done, double *src, double *gain,
                     const int32_t *mdeg, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  mp_tables_kernel<<<B, 256, 0, st>>>(B, k, m, theta, win, lock, done, src, gain, mdeg);
  return hipGetLastError();
}

__global__ void mp_prep_kernel(int B, int64_t n, int64_t ld, int64_t bs, int32_t k,
                               const int32_t *__restrict__ lock, const double *__restrict__ X,
                               const double *__restrict__ W, const double *__restrict__ theta,
                               const double *__restrict__ coef, float *__restrict__ R32,
                               float *__restrict__ E1) {
  const int b = blockIdx.z;
  const int c = (lock ? lock[b] : 0) + blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k || p >= n) return;
  const int64_t o = (int64_t)b * bs + (int64_t)c * ld + p;
  const double r = W[o] - theta[(int64_t)b * k + c] * X[o];
  R32[o] = (float)r;
  E1[o] = (float)(coef[3 * b + 0] * r);               // step-0 coefficient sigma_1 / e
}

hipError_t mp_prep(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, const int32_t *lock,
                   const double *X, const double *W, const double *theta, const double *coef,
                   float *R32, float *E1, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  mp_prep_kernel<<<dim3((unsigned)ceil_div(n, 256), k, B), 256, 0, st>>>(B, n, ld, bs, k, lock, X,
                                                                         W, theta, coef, R32, E1);
  return hipGetLastError();
}

__global__ void mp_final_kernel(int64_t n, int64_t ld, int64_t bs, int32_t k,
                                const int32_t *__restrict__ lock, const double *__restrict__ X,
                                const float *__restrict__ Em, const double *__restrict__ gain,
                                double *__restrict__ Y) {
  const int b = blockIdx.z;
  const int c = (lock ? lock[b] : 0) + blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k || p >= n) return;
  const int64_t o = (int64_t)b * bs + (int64_t)c * ld + p;
  Y[o] = X[o] * gain[(int64_t)b * k + c] + (double)Em[o];
}

hipError_t mp_final(int B, int64_t n, int64_t ld, int64_t bs, int32_t k, const int32_t *lock,
                    const double *X, const float *Em, const double *gain, double *Y,
                    hipStream_t st) {
  if (B <= 0) return hipSuccess;
  mp_final_kernel<<<dim3((unsigned)ceil_div(n, 256), k, B), 256, 0, st>>>(n, ld, bs, k, lock, X, Em,
                                                                          gain, Y);
  return hipGetLastError();
}

// Warm start across grid sides: column c of X is a nodal field on the N0 x N0 interior grid
// of the unit square (node (iy, ix) at ((ix+1)/(N0+1), (iy+1)/(N0+1)), entry iy*N0 + ix, zero
// on the boundary); Y column c is its bilinear interpolant at the N1 x N1 nodes.  The source
// position of output node i is (i+1)(N0+1)/(N1+1) - 1 in units of the source spacing.
// grid (ceil(N1^2 / 256), ncols): one thread per output node and column.
__global__ void __launch_bounds__(256) interp_kernel(int32_t N0, int32_t N1,
                                                     const double *__restrict__ X, int64_t ldx,
                                                     double *__restrict__ Y, int64_t ldy) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)N1 * N1) return;
  const int oy = (int)(p / N1), ox = (int)(p - (int64_t)oy * N1);
  const double *x = X + (int64_t)blockIdx.y * ldx;
  const double sy = (double)((int64_t)(oy + 1) * (N0 + 1)) / (double)(N1 + 1) - 1.0;
  const double sx = (double)((int64_t)(ox + 1) * (N0 + 1)) / (double)(N1 + 1) - 1.0;
  const int jy = (int)floor(sy), jx = (int)floor(sx);
  const double fy = sy - jy, fx = sx - jx;
  auto at = [&](int iy, int ix) -> double {
    return (iy >= 0 && iy < N0 && ix >= 0 && ix < N0) ? x[(int64_t)iy * N0 + ix] : 0.0;
  };
  const double lo = (1.0 - fx) * at(jy, jx) + fx * at(jy, jx + 1);
  const double hi = (1.0 - fx) * at(jy + 1, jx) + fx * at(jy + 1, jx + 1);
  Y[(int64_t)blockIdx.y * ldy + p] = (1.0 - fy) * lo + fy * hi;
}

hipError_t interpolate_fields(int32_t N0, int32_t N1, int32_t ncols, const double *X,
                              int64_t ldx, double *Y, int64_t ldy, hipStream_t st) {
  if (ncols <= 0 || N1 <= 0) return hipSuccess;
  interp_kernel<<<dim3((unsigned)ceil_div((int64_t)N1 * N1, 256), (unsigned)ncols), 256, 0, st>>>(
      N0, N1, X, ldx, Y, ldy);
  return hipGetLastError();
}

// Adaptive filter degrees for the next outer iteration (the optimized filter cited for
// Algorithm 1): with the window the next iteration will use (as in cheb_kernel: c, e from the
// smallest and largest Ritz values and beta), an active column with Ritz value theta and
// residual r needs m = ceil(ln(r / tol) / ln|rho|) steps, |rho| = |t| + sqrt(t^2 - 1),
// t = (theta - c) / e; clamped to [mlo, mhi] (mhi when |t| <= 1).  mdeg[b] = the largest.
// grid B, 256 threads.
__global__ void __launch_bounds__(256) adaptive_degree_kernel(
    int32_t k, const int32_t *__restrict__ lock, const int32_t *__restrict__ done,
    const double *__restrict__ theta, const double *__restrict__ res,
    const double *__restrict__ bnd, double tol, int32_t mlo, int32_t mhi,
    int32_t *__restrict__ cdeg, int32_t *__restrict__ mdeg) {
  __shared__ int32_t smax[4];
  const int b = blockIdx.x;
  if (done[b]) return;
  const double lam = theta[(int64_t)b * k], alpha0 = theta[(int64_t)b * k + k - 1];
  double alpha = alpha0, beta = bnd[b * 4 + 3];
  const double span = fmax(fabs(alpha), fabs(lam));
  if (!(beta > alpha + 1e-12 * span)) beta = alpha + fmax(1e-3 * span, 1e-300);
  const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
  int32_t best = mlo;
  for (int col = lock[b] + threadIdx.x; col < k; col += blockDim.x) {
    const double t = (theta[(int64_t)b * k + col] - c) / e;
    int32_t m = mhi;
    if (fabs(t) > 1.0) {
      const double rho = fabs(t) + sqrt(t * t - 1.0);
      const double r = fmax(res[(int64_t)b * k + col], tol);
      const double need = ceil(log(r / tol) / log(rho) - 1e-12);
      m = (int32_t)fmin((double)mhi, fmax((double)mlo, need));
    }
    cdeg[(int64_t)b * k + col] = m;
    best = max(best, m);
  }
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_down(best, o, 64));
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = smax[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, smax[w]);
    mdeg[b] = m;
  }
}

// P = b_s X + g_s Z (Z optional) on the active columns and the first rows[b] rows of every
// problem: the non-operator terms of a square-mode filter step, coef = that step's (a, b, g).
__global__ void axpby_kernel(int64_t ld, int64_t bs, int32_t k, const int32_t *__restrict__ lock,
                             const double *__restrict__ X, const double *__restrict__ Z,
                             const double *__restrict__ coef, double *__restrict__ P,
                             const int32_t *__restrict__ rows) {
  const int b = blockIdx.z;
  const int32_t l = lock[b];
  const int c = l + (int)blockIdx.y;
  if (c >= k) return;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= rows[b]) return;
  const int64_t o = (int64_t)b * bs + (int64_t)c * ld + p;
  const double bc = coef[3 * b + 1], g = coef[3 * b + 2];
  P[o] = Z ? bc * X[o] + g * Z[o] : bc * X[o];
}

hipError_t axpby_active(int B, int64_t nmax, int64_t ld, int64_t bs, int32_t k,
                        const int32_t *lock, const double *X, const double *Z, const double *coef,
                        double *P, const int32_t *rows, hipStream_t st) {
  if (B <= 0 || nmax <= 0 || k <= 0) return hipSuccess;
  axpby_kernel<<<dim3((unsigned)ceil_div(nmax, 256), (unsigned)k, (unsigned)B), 256, 0, st>>>(
      ld, bs, k, lock, X, Z, coef, P, rows);
  return hipGetLastError();
}

// Reorder the active Ritz pairs of every problem by |theta| (stable: equal magnitudes keep
// the ascending order the eigensolver gave): theta in place, Z (active columns, ldm x ldm
// per problem) into Zout.
__global__ void __launch_bounds__(256) magnitude_order_kernel(
    int32_t k, const int32_t *__restrict__ lock, double *__restrict__ theta,
    const double *__restrict__ Z, double *__restrict__ Zout, int32_t ldm) {
  __shared__ double th[kMaxK];
  __shared__ int perm[kMaxK];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int32_t l = lock[b];
  const int ka = k - l;
  if (ka <= 0) return;
  for (int j = tid; j < ka; j += 256) th[j] = theta[(int64_t)b * k + l + j];
  __syncthreads();
  for (int j = tid; j < ka; j += 256) {
    const double aj = fabs(th[j]);
    int r = 0;
    for (int i = 0; i < ka; ++i) {
      const double ai = fabs(th[i]);
      r += (ai < aj || (ai == aj && i < j)) ? 1 : 0;
    }
    perm[r] = j;
  }
  __syncthreads();
  for (int j = tid; j < ka; j += 256) theta[(int64_t)b * k + l + j] = th[perm[j]];
  const double *Zb = Z + (int64_t)b * ldm * ldm;
  double *Ob = Zout + (int64_t)b * ldm * ldm;
  for (int e = tid; e < ka * ka; e += 256) {
    const int r = e % ka, j = e / ka;
    Ob[r + (int64_t)j * ldm] = Zb[r + (int64_t)perm[j] * ldm];
  }
}

hipError_t magnitude_order(int B, int32_t k, const int32_t *lock, double *theta, const double *Z,
                           double *Zout, int32_t ldm, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  magnitude_order_kernel<<<B, 256, 0, st>>>(k, lock, theta, Z, Zout, ldm);
  return hipGetLastError();
}

hipError_t adaptive_degrees(int B, int32_t k, const int32_t *lock, const int32_t *done,
                            const double *theta, const double *res, const double *bnd,
                            double tol, int32_t mlo, int32_t mhi, int32_t *cdeg, int32_t *mdeg,
                            hipStream_t st) {
  if (B <= 0) return hipSuccess;
  adaptive_degree_kernel<<<B, 256, 0, st>>>(k, lock, done, theta, res, bnd, tol, mlo, mhi, cdeg,
                                            mdeg);
  return hipGetLastError();
}

}  // namespace scsf
