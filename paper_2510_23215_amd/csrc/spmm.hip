// Operator application and the Chebyshev three-term step on a block of vectors (gfx950).
//
// One step of the scaled recurrence of Algorithm 1 (Section 2.2) is
//   Y_{i+1} = a (A Y_i) + b Y_i + g Y_{i-1},
// with a = 2 sigma_{i+1} / e, b = -2 sigma_{i+1} c / e, g = -sigma_i sigma_{i+1} (a = sigma_1/e,
// b = -sigma_1 c / e, g = 0 for the first step).  The kernel streams the block once: each
// thread owns one grid node and CPT consecutive columns, so the node's stencil coefficients
// are loaded once and reused across the columns, and the loads of a wavefront are
// contiguous in every column (column-major blocks).  Neighbour values along x come from the
// same cache lines; the +-N neighbours are re-read from L2 by the adjacent row tiles.
#include "stencil.h"

namespace scsf {

// T = double: the plain FP64 step.  T = float (mixed precision): the same step on the FP32
// correction block E, with the source term src[b*k + c] * R[:, c] of the residual form of the
// recurrence (see mp_* in misc.hip); the operator coefficients are read in FP64 and rounded.
template <int KIND, int CPT, typename T, bool SRC>
__global__ void __launch_bounds__(256) spmm_step_kernel(
    const OpDev *__restrict__ ops, const T *__restrict__ X, const T *__restrict__ Z,
    T *__restrict__ Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
    const int32_t *__restrict__ lock, const double *__restrict__ coef, int has_z,
    const T *__restrict__ R, const double *__restrict__ src, const int32_t *__restrict__ mdeg,
    int32_t step) {
  const int b = blockIdx.z;
  if (mdeg && step >= mdeg[b]) return;                // this problem's filter has finished
  const OpDev op = ops[b];
  const int64_t n = op.n;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t c0, cnt;
  col_range(mode, k, lock, b, c0, cnt);
  const int j0 = blockIdx.y * CPT;
  if (p >= n || j0 >= cnt) return;
  const T a = (T)coef[3 * b + 0], bc = (T)coef[3 * b + 1], g = (T)coef[3 * b + 2];
  const int64_t off = (int64_t)b * bs + (int64_t)(c0 + j0) * ld;
  const T *x = X + off;
  T *y = Y + off;
  const T *z = has_z ? Z + off : nullptr;
  const int jn = min(CPT, cnt - j0);
  T sj[CPT];
  if constexpr (SRC) {
#pragma unroll
    for (int j = 0; j < CPT; ++j) sj[j] = (j < jn) ? (T)src[(int64_t)b * k + c0 + j0 + j] : (T)0;
  }

  if constexpr (KIND == SCSF_STENCIL5) {
    const int N = op.N;
    const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
    const double cw64 = op.wx[(int64_t)iy * (N + 1) + ix];
    const double ce64 = op.wx[(int64_t)iy * (N + 1) + ix + 1];
    const double cs64 = op.wy[(int64_t)iy * N + ix];
    const double cn64 = op.wy[(int64_t)(iy + 1) * N + ix];
    const T cd = (T)(cw64 + ce64 + cs64 + cn64 + (op.v ? op.v[p] : 0.0));
    const T cw = (T)cw64, ce = (T)ce64, cs = (T)cs64, cn = (T)cn64;
    const bool hw = ix > 0, he = ix < N - 1, hs = iy > 0, hn = iy < N - 1;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (j < jn) {
        const T *xc = x + (int64_t)j * ld;
        const T xv = xc[p];
        T ax = cd * xv;
        if (hw) ax -= cw * xc[p - 1];
        if (he) ax -= ce * xc[p + 1];
        if (hs) ax -= cs * xc[p - N];
        if (hn) ax -= cn * xc[p + N];
        T r = a * ax + bc * xv;
        if (z) r += g * z[(int64_t)j * ld + p];
        if constexpr (SRC) r += sj[j] * R[off + (int64_t)j * ld + p];
        y[(int64_t)j * ld + p] = r;
      }
    }
  } else if constexpr (KIND == SCSF_STENCIL9) {
    const int N = op.N;
    const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
    double c64[9];
    stencil9_coeffs(op, iy, ix, c64);
    T c9[9];
    bool ok[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      c9[t] = (T)c64[t];
      ok[t] = (iy + dy >= 0) && (iy + dy < N) && (ix + dx >= 0) && (ix + dx < N);
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (j < jn) {
        const T *xc = x + (int64_t)j * ld;
        const T xv = xc[p];
        T ax = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int dy = t / 3 - 1, dx = t % 3 - 1;
          if (ok[t]) ax += c9[t] * xc[p + dy * N + dx];
        }
        T r = a * ax + bc * xv;
        if (z) r += g * z[(int64_t)j * ld + p];
        if constexpr (SRC) r += sj[j] * R[off + (int64_t)j * ld + p];
        y[(int64_t)j * ld + p] = r;
      }
    }
  } else {  // CSR
    const int32_t r0 = op.row_ptr[p], r1 = op.row_ptr[p + 1];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (j < jn) {
        const T *xc = x + (int64_t)j * ld;
        T ax = 0;
        for (int32_t q = r0; q < r1; ++q) ax += (T)op.val[q] * xc[op.col_idx[q]];
        T r = a * ax + bc * xc[p];
        if (z) r += g * z[(int64_t)j * ld + p];
        if constexpr (SRC) r += sj[j] * R[off + (int64_t)j * ld + p];
        y[(int64_t)j * ld + p] = r;
      }
    }
  }
}

template <int CPT, typename T, bool SRC>
static void launch_kind(const OpDev *ops, int B, int32_t kind, int64_t nmax, const T *X,
                        const T *Z, T *Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                        const int32_t *lock, const double *coef, int hz, const T *R,
                        const double *src, const int32_t *mdeg, int32_t step, hipStream_t st) {
  dim3 block(256);
  dim3 grid((unsigned)ceil_div(nmax, 256), (unsigned)ceil_div(k, CPT), (unsigned)B);
  if (kind == SCSF_STENCIL5)
    spmm_step_kernel<SCSF_STENCIL5, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step);
  else if (kind == SCSF_STENCIL9)
    spmm_step_kernel<SCSF_STENCIL9, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step);
  else
    spmm_step_kernel<SCSF_CSR, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step);
}

// cpt: columns per thread (2, 4 or 8), the tile the autotuner chooses per (n, k).
template <typename T, bool SRC>
static hipError_t launch_step(const OpDev *ops, int B, int32_t kind, int64_t nmax, const T *X,
                              const T *Z, T *Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                              const int32_t *lock, const double *coef, bool has_z, const T *R,
                              const double *src, const int32_t *mdeg, int32_t step, int cpt,
                              hipStream_t st) {
  if (B <= 0 || nmax <= 0 || k <= 0) return hipSuccess;
  const int hz = has_z ? 1 : 0;
  if (cpt == 2)
    launch_kind<2, T, SRC>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src,
                           mdeg, step, st);
  else if (cpt == 8)
    launch_kind<8, T, SRC>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src,
                           mdeg, step, st);
  else
    launch_kind<4, T, SRC>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src,
                           mdeg, step, st);
  return hipGetLastError();
}

hipError_t spmm_step(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t /*Nmax*/,
                     const double *X, const double *Z, double *Y, int64_t ld, int64_t bs,
                     int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                     bool has_z, hipStream_t st, const int32_t *mdeg, int32_t step, int cpt) {
  return launch_step<double, false>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                    has_z, nullptr, nullptr, mdeg, step, cpt, st);
}

hipError_t spmm_step32(const OpDev *ops, int B, int32_t kind, int64_t nmax, const float *X,
                       const float *Z, float *Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                       const int32_t *lock, const double *coef, bool has_z, const float *R,
                       const double *src, hipStream_t st, const int32_t *mdeg, int32_t step,
                       int cpt) {
  if (R)
    return launch_step<float, true>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                    has_z, R, src, mdeg, step, cpt, st);
  return launch_step<float, false>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   has_z, nullptr, nullptr, mdeg, step, cpt, st);
}

}  // namespace scsf
