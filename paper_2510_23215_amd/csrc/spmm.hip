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

#include <type_traits>

namespace scsf {

// Per-column degree (adaptive filter): column c of problem b takes part in the step while
// step < its degree, raised by at most 2 to the residue of the iteration's degree mtot mod 3
// so that every column ends in the same buffer of the three-buffer ring.
__device__ inline bool column_active(const int32_t *cdeg, int32_t mtot, int32_t step, int b,
                                     int32_t k, int c) {
  if (!cdeg) return true;
  int32_t d = cdeg[(int64_t)b * k + c];
  d += ((mtot - d) % 3 + 3) % 3;
  return step < d;
}

// T = double: the plain FP64 step.  T = float (mixed precision): the same step on the FP32
// correction block E, with the source term src[b*k + c] * R[:, c] of the residual form of the
// recurrence (see mp_* in misc.hip); the operator coefficients are read in FP64 and rounded.
template <int KIND, int CPT, typename T, bool SRC>
__global__ void __launch_bounds__(256) spmm_step_kernel(
    const OpDev *__restrict__ ops, const T *__restrict__ X, const T *__restrict__ Z,
    T *__restrict__ Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
    const int32_t *__restrict__ lock, const double *__restrict__ coef, int has_z,
    const T *__restrict__ R, const double *__restrict__ src, const int32_t *__restrict__ mdeg,
    int32_t step, const int32_t *__restrict__ cdeg, int32_t mtot) {
  // XCD-aware order: the hardware deals workgroups to the 8 XCDs round-robin by linear id, and
  // each XCD has its own L2.  Remapping the linear id gives every XCD one contiguous range of
  // row tiles (of one problem and column group), so the +-N neighbour rows a tile reads were
  // just fetched by its neighbour tile on the same XCD.
  const uint32_t gx = gridDim.x, gy = gridDim.y, total = gx * gy * gridDim.z;
  uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t per = total / 8;
  if (lin < 8 * per) lin = (lin % 8) * per + lin / 8;
  const uint32_t tile = lin % gx, rest = lin / gx;
  const int b = (int)(rest / gy);
  if (mdeg && step >= mdeg[b]) return;                // this problem's filter has finished
  const OpDev op = ops[b];
  const int64_t n = op.n;
  const int64_t p = (int64_t)tile * blockDim.x + threadIdx.x;
  int32_t c0, cnt;
  col_range(mode, k, lock, b, c0, cnt);
  const int j0 = (int)(rest % gy) * CPT;
  if (p >= n || j0 >= cnt) return;
  const T a = (T)coef[3 * b + 0], bc = (T)coef[3 * b + 1], g = (T)coef[3 * b + 2];
  const int64_t off = (int64_t)b * bs + (int64_t)(c0 + j0) * ld;
  const T *x = X + off;
  T *y = Y + off;
  const T *z = has_z ? Z + off : nullptr;
  const int jn = min(CPT, cnt - j0);
  bool act[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) act[j] = j < jn && column_active(cdeg, mtot, step, b, k, c0 + j0 + j);
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
      if (act[j]) {
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
      if (act[j]) {
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
      if (act[j]) {
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

// LDS-staged step for the grid stencils: a workgroup takes TILE = 256 NPT consecutive nodes and
// CPT columns.  It stages each column's nodes [p0 - H, p0 + TILE + H) (H = N, or N + 1 for the
// 9-point stencil) into LDS with coalesced loads, then every thread computes NPT nodes
// (p0 + t 256 + tid, so the Z reads and Y writes of a wavefront stay contiguous) from LDS.
// Each element of X is read from HBM about once (the 2H halo nodes come from L2), and the
// memory instructions per node and column drop fourfold against the register form above.
// One node's step for JN columns staged in LDS (JN = CPT on full column groups, so every
// loop below unrolls without per-column checks).
// KIND: SCSF_STENCIL5 (no problem of the batch has a potential: no per-node branch),
// kStencil5V (5-point, potential where op.v is set) or SCSF_STENCIL9.
constexpr int kStencil5V = 105;
constexpr size_t kFusedBytes = 65536;                 // dynamic LDS of one fused workgroup

// Z (the block two steps back) and Y are touched once per step: streamed with non-temporal
// loads and stores, so they do not displace the staged tiles' halos and coefficients from L2.
template <int KIND, int JN, typename T, bool SRC, bool HZ>
__device__ inline void lds_node(const OpDev &op, const T *sx, int span, int e, int64_t p,
                                int N, T a, T bc, T g, const T *srcj,
                                const T *__restrict__ Z, const T *__restrict__ R,
                                T *__restrict__ Y, int64_t off, int64_t ld) {
  const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
  if constexpr (KIND == SCSF_STENCIL5 || KIND == kStencil5V) {
    const double cw64 = op.wx[(int64_t)iy * (N + 1) + ix];
    const double ce64 = op.wx[(int64_t)iy * (N + 1) + ix + 1];
    const double cs64 = op.wy[(int64_t)iy * N + ix];
    const double cn64 = op.wy[(int64_t)(iy + 1) * N + ix];
    double vp = 0.0;
    if constexpr (KIND == kStencil5V) vp = op.v ? op.v[p] : 0.0;
    const T cd = (T)(cw64 + ce64 + cs64 + cn64 + vp);
    const T mw = ix > 0 ? (T)cw64 : (T)0, me = ix < N - 1 ? (T)ce64 : (T)0;
    const T ms = iy > 0 ? (T)cs64 : (T)0, mn = iy < N - 1 ? (T)cn64 : (T)0;
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const T *sj = sx + j * span;
      const T xv = sj[e];
      const T ax = cd * xv - mw * sj[e - 1] - me * sj[e + 1] - ms * sj[e - N] - mn * sj[e + N];
      const int64_t o = off + (int64_t)j * ld + p;
      T r = a * ax + bc * xv;
      if constexpr (HZ) r += g * __builtin_nontemporal_load(&Z[o]);
      if constexpr (SRC) r += srcj[j] * R[o];
      __builtin_nontemporal_store(r, &Y[o]);
    }
  } else {
    double c64[9];
    stencil9_coeffs(op, iy, ix, c64);
    T c9[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int dy = q / 3 - 1, dx = q % 3 - 1;
      const bool ok = (iy + dy >= 0) && (iy + dy < N) && (ix + dx >= 0) && (ix + dx < N);
      c9[q] = ok ? (T)c64[q] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const T *sj = sx + j * span;
      T ax = 0;
#pragma unroll
      for (int q = 0; q < 9; ++q) ax += c9[q] * sj[e + (q / 3 - 1) * N + (q % 3 - 1)];
      const int64_t o = off + (int64_t)j * ld + p;
      T r = a * ax + bc * sj[e];
      if constexpr (HZ) r += g * __builtin_nontemporal_load(&Z[o]);
      if constexpr (SRC) r += srcj[j] * R[o];
      __builtin_nontemporal_store(r, &Y[o]);
    }
  }
}

// LDS-staged step for the grid stencils: a workgroup takes TILE = 256 NPT consecutive nodes and
// CPT columns.  It stages each column's nodes [p0 - H, p0 + TILE + H) (H = N, or N + 1 for the
// 9-point stencil) into LDS with coalesced loads, then every thread computes NPT nodes
// (p0 + t 256 + tid, so the Z reads and Y writes of a wavefront stay contiguous) from LDS.
// Each element of X is read from HBM about once (the 2H halo nodes come from L2), and the
// memory instructions per node and column drop fourfold against the register form above.
template <int KIND, int CPT, int NPT, typename T, bool SRC, bool HZ>
__global__ void __launch_bounds__(256) spmm_lds_kernel(
    const OpDev *__restrict__ ops, const T *__restrict__ X, const T *__restrict__ Z,
    T *__restrict__ Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
    const int32_t *__restrict__ lock, const double *__restrict__ coef,
    const T *__restrict__ R, const double *__restrict__ src, const int32_t *__restrict__ mdeg,
    int32_t step, const int32_t *__restrict__ cdeg, int32_t mtot) {
  constexpr int TILE = 256 * NPT;
  extern __shared__ unsigned char smem_raw[];
  T *sx = reinterpret_cast<T *>(smem_raw);
  const int b = blockIdx.z;
  if (mdeg && step >= mdeg[b]) return;
  const OpDev op = ops[b];
  const int N = op.N;
  const int64_t n = op.n;
  const int64_t p0 = (int64_t)blockIdx.x * TILE;
  if (p0 >= n) return;
  int32_t c0, cnt;
  col_range(mode, k, lock, b, c0, cnt);
  const int j0 = blockIdx.y * CPT;
  if (j0 >= cnt) return;
  const int jn = min(CPT, cnt - j0);
  bool act[CPT];
  bool any = false, all = true;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    act[j] = j < jn && column_active(cdeg, mtot, step, b, k, c0 + j0 + j);
    any = any || act[j];
    all = all && act[j];
  }
  if (!any) return;                                   // every column of the group has stopped
  const int H = (KIND == SCSF_STENCIL9) ? N + 1 : N;
  const int span = TILE + 2 * H;
  const int tid = threadIdx.x;
  const int64_t off = (int64_t)b * bs + (int64_t)(c0 + j0) * ld;
  const T *xb = X + off;
  // U rows of 256 nodes per pass, every load of a pass issued before the first LDS store:
  // each thread keeps U * CPT loads in flight instead of CPT
  constexpr int U = 4;
  for (int e0 = tid; e0 < span; e0 += 256 * U) {
    T v[U][CPT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      const int64_t q = p0 - H + e;
      const bool in = e < span && q >= 0 && q < n;
#pragma unroll
      for (int j = 0; j < CPT; ++j) v[u][j] = (act[j] && in) ? xb[(int64_t)j * ld + q] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      if (e < span) {
#pragma unroll
        for (int j = 0; j < CPT; ++j)
          if (act[j]) sx[j * span + e] = v[u][j];
      }
    }
  }
  __syncthreads();
  const T a = (T)coef[3 * b + 0], bc = (T)coef[3 * b + 1], g = (T)coef[3 * b + 2];
  T srcj[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j)
    srcj[j] = (SRC && j < jn) ? (T)src[(int64_t)b * k + c0 + j0 + j] : (T)0;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int64_t p = p0 + t * 256 + tid;
    if (p >= n) break;
    const int e = H + t * 256 + tid;
    if (all) {
      lds_node<KIND, CPT, T, SRC, HZ>(op, sx, span, e, p, N, a, bc, g, srcj, Z, R, Y, off, ld);
    } else {
      // a partial column group, or columns past their degree (indices stay compile-time)
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        if (act[j]) {
          const T one[1] = {srcj[j]};
          lds_node<KIND, 1, T, SRC, HZ>(op, sx + j * span, span, e, p, N, a, bc, g, one, Z, R, Y,
                                        off + (int64_t)j * ld, ld);
        }
      }
    }
  }
}

// S Chebyshev steps in one pass over the block (temporal blocking of the grid stencils).
// A workgroup takes TILE = 256 NPT consecutive nodes and CPT columns.  It stages level i
// (Xc) on the tile +- S H nodes and level i-1 (Xp) on the tile +- (S-1) H (H = N, or N + 1
// for the 9-point stencil) in two LDS arrays per column, then runs the S steps in LDS: step
// t computes level i+t+1 on the tile +- (S-t-1) H, each node from its neighbours in the
// newest level and its own value in the one before, and writes it over that older value
// (only the node itself reads it), so two arrays carry all levels.  The last two levels are
// written to Ocur (level i+S) and Oprev (level i+S-1).  HBM traffic per column and node:
// two reads and two writes for S steps, against three per step for the single-step kernel;
// the halos come from L2 (neighbouring tiles read the same rows).  Nodes outside the grid are
// zero in every level (Dirichlet).  coef holds the S steps' (a, b, g), step t at
// coef[(t B + b) 3]; with HZ false (i = 0) there is no level -1 and the first g is 0.
// Problems with mdeg[b] <= i have finished (the degrees are aligned to the groups).
template <int KIND, int CPT, int NPT, int S, bool HZ>
__global__ void __launch_bounds__(256) spmm_fused_kernel(
    const OpDev *__restrict__ ops, int B, const double *__restrict__ Xc,
    const double *__restrict__ Xp, double *__restrict__ Ocur, double *__restrict__ Oprev,
    int64_t ld, int64_t bs, int32_t mode, int32_t k, const int32_t *__restrict__ lock,
    const double *__restrict__ coef, const int32_t *__restrict__ mdeg, int32_t step0) {
  constexpr int TILE = 256 * NPT;
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.z;
  if (mdeg && step0 >= mdeg[b]) return;
  const OpDev op = ops[b];
  const int N = op.N;
  const int64_t n = op.n;
  const int64_t p0 = (int64_t)blockIdx.x * TILE;
  if (p0 >= n) return;
  int32_t c0, cnt;
  col_range(mode, k, lock, b, c0, cnt);
  const int j0 = blockIdx.y * CPT;
  if (j0 >= cnt) return;
  const int jn = min(CPT, cnt - j0);
  const int H = (KIND == SCSF_STENCIL9) ? N + 1 : N;
  const int span = TILE + 2 * S * H;
  double *la = reinterpret_cast<double *>(smem_raw);          // CPT columns x span
  double *lb = la + (size_t)CPT * span;                        // CPT columns x span
  const int tid = threadIdx.x;
  const int64_t base = p0 - (int64_t)S * H;                    // node of LDS entry 0
  const int64_t off = (int64_t)b * bs + (int64_t)(c0 + j0) * ld;
  // stage level i into la (whole span) and level i-1 into lb (span less H at each end)
  constexpr int U = 4;
  for (int e0 = tid; e0 < span; e0 += 256 * U) {
    double v[U][CPT], w[U][CPT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      const int64_t q = base + e;
      const bool in = e < span && q >= 0 && q < n;
      const bool inz = HZ && in && e >= H && e < span - H;
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        v[u][j] = (j < jn && in) ? Xc[off + (int64_t)j * ld + q] : 0.0;
        w[u][j] = (j < jn && inz) ? Xp[off + (int64_t)j * ld + q] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 256;
      if (e < span) {
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          la[j * span + e] = v[u][j];
          lb[j * span + e] = w[u][j];
        }
      }
    }
  }
  __syncthreads();
  double *cur = la, *prv = lb;
#pragma unroll 1
  for (int t = 0; t < S; ++t) {
    const double a = coef[((int64_t)t * B + b) * 3 + 0];
    const double bc = coef[((int64_t)t * B + b) * 3 + 1];
    const double g = coef[((int64_t)t * B + b) * 3 + 2];
    const int lo = (t + 1) * H, hi = span - (t + 1) * H;
    for (int e = lo + tid; e < hi; e += 256) {
      const int64_t q = base + e;
      if (q < 0 || q >= n) {
#pragma unroll
        for (int j = 0; j < CPT; ++j) prv[j * span + e] = 0.0;
        continue;
      }
      const int iy = (int)(q / N), ix = (int)(q - (int64_t)iy * N);
      if constexpr (KIND == SCSF_STENCIL5 || KIND == kStencil5V) {
        const double cw = op.wx[(int64_t)iy * (N + 1) + ix];
        const double ce = op.wx[(int64_t)iy * (N + 1) + ix + 1];
        const double cs = op.wy[(int64_t)iy * N + ix];
        const double cn = op.wy[(int64_t)(iy + 1) * N + ix];
        double vp = 0.0;
        if constexpr (KIND == kStencil5V) vp = op.v ? op.v[q] : 0.0;
        const double cd = cw + ce + cs + cn + vp;
        const double mw = ix > 0 ? cw : 0.0, me = ix < N - 1 ? ce : 0.0;
        const double ms = iy > 0 ? cs : 0.0, mn = iy < N - 1 ? cn : 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          const double *cj = cur + j * span;
          const double xv = cj[e];
          const double ax = cd * xv - mw * cj[e - 1] - me * cj[e + 1] - ms * cj[e - N] -
                            mn * cj[e + N];
          double r = a * ax + bc * xv;
          if (HZ || t > 0) r += g * prv[j * span + e];
          prv[j * span + e] = r;
        }
      } else {
        double c64[9], c9[9];
        stencil9_coeffs(op, iy, ix, c64);
        // a select into a second array: with the conditional store `if (!ok) c64[qq] = 0`
        // hipcc dropped the zeroing of the (-1, -1) coefficient at ix = 0, so the left-edge
        // nodes picked up the previous row's last node
#pragma unroll
        for (int qq = 0; qq < 9; ++qq) {
          const int dy = qq / 3 - 1, dx = qq % 3 - 1;
          const bool ok = (iy + dy >= 0) && (iy + dy < N) && (ix + dx >= 0) && (ix + dx < N);
          c9[qq] = ok ? c64[qq] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          const double *cj = cur + j * span;
          double ax = 0.0;
#pragma unroll
          for (int qq = 0; qq < 9; ++qq) ax += c9[qq] * cj[e + (qq / 3 - 1) * N + (qq % 3 - 1)];
          double r = a * ax + bc * cj[e];
          if (HZ || t > 0) r += g * prv[j * span + e];
          prv[j * span + e] = r;
        }
      }
    }
    __syncthreads();
    double *tmp = cur;
    cur = prv;
    prv = tmp;
  }
  // cur: level i+S, prv: level i+S-1, valid on the tile
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int64_t q = p0 + u * 256 + tid;
    if (q >= n) break;
    const int e = S * H + u * 256 + tid;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (j < jn) {
        const int64_t o = off + (int64_t)j * ld + q;
        __builtin_nontemporal_store(cur[j * span + e], &Ocur[o]);
        __builtin_nontemporal_store(prv[j * span + e], &Oprev[o]);
      }
    }
  }
}

template <int CPT, int NPT, int S>
static bool launch_fused_t(const OpDev *ops, int B, int32_t kind, bool pot, int64_t nmax,
                           int32_t Nmax, const double *Xc, const double *Xp, double *Ocur,
                           double *Oprev, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                           const int32_t *lock, const double *coef, const int32_t *mdeg,
                           int32_t step0, hipStream_t st) {
  constexpr int TILE = 256 * NPT;
  const int64_t H = (kind == SCSF_STENCIL9) ? (int64_t)Nmax + 1 : Nmax;
  const size_t shm = (size_t)2 * CPT * (TILE + 2 * S * H) * sizeof(double);
  if (shm > kFusedBytes) return false;
  dim3 grid((unsigned)ceil_div(nmax, TILE), (unsigned)ceil_div(k, CPT), (unsigned)B);
  const bool hz = Xp != nullptr;
  auto go = [&](auto kern) {
    kern<<<grid, 256, shm, st>>>(ops, B, Xc, Xp, Ocur, Oprev, ld, bs, mode, k, lock, coef, mdeg,
                                 step0);
  };
  if (kind == SCSF_STENCIL5 && !pot) {
    if (hz) go(spmm_fused_kernel<SCSF_STENCIL5, CPT, NPT, S, true>);
    else go(spmm_fused_kernel<SCSF_STENCIL5, CPT, NPT, S, false>);
  } else if (kind == SCSF_STENCIL5) {
    if (hz) go(spmm_fused_kernel<kStencil5V, CPT, NPT, S, true>);
    else go(spmm_fused_kernel<kStencil5V, CPT, NPT, S, false>);
  } else {
    if (hz) go(spmm_fused_kernel<SCSF_STENCIL9, CPT, NPT, S, true>);
    else go(spmm_fused_kernel<SCSF_STENCIL9, CPT, NPT, S, false>);
  }
  return true;
}

template <int S>
static bool launch_fused_s(int tile, const OpDev *ops, int B, int32_t kind, bool pot,
                           int64_t nmax, int32_t Nmax, const double *Xc, const double *Xp,
                           double *Ocur, double *Oprev, int64_t ld, int64_t bs, int32_t mode,
                           int32_t k, const int32_t *lock, const double *coef,
                           const int32_t *mdeg, int32_t step0, hipStream_t st) {
  // tile: columns per thread (1, 2, 4) with 4 nodes per thread; a smaller tile when the
  // LDS arrays of the larger do not fit
  if (tile >= 4 && launch_fused_t<4, 4, S>(ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld,
                                           bs, mode, k, lock, coef, mdeg, step0, st))
    return true;
  if (tile >= 2 && launch_fused_t<2, 4, S>(ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld,
                                           bs, mode, k, lock, coef, mdeg, step0, st))
    return true;
  return launch_fused_t<1, 4, S>(ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld, bs, mode,
                                 k, lock, coef, mdeg, step0, st);
}

template <int CPT, typename T, bool SRC>
static void launch_reg(const OpDev *ops, int B, int32_t kind, int64_t nmax, const T *X,
                       const T *Z, T *Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                       const int32_t *lock, const double *coef, int hz, const T *R,
                       const double *src, const int32_t *mdeg, int32_t step,
                       const int32_t *cdeg, int32_t mtot, hipStream_t st) {
  dim3 block(256);
  dim3 grid((unsigned)ceil_div(nmax, 256), (unsigned)ceil_div(k, CPT), (unsigned)B);
  if (kind == SCSF_STENCIL5)
    spmm_step_kernel<SCSF_STENCIL5, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step, cdeg, mtot);
  else if (kind == SCSF_STENCIL9)
    spmm_step_kernel<SCSF_STENCIL9, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step, cdeg, mtot);
  else
    spmm_step_kernel<SCSF_CSR, CPT, T, SRC><<<grid, block, 0, st>>>(
        ops, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src, mdeg, step, cdeg, mtot);
}

constexpr size_t kStageBytes = 65536;                 // dynamic LDS of one staged workgroup

// Thin-plate step: A = S L diag(D) L S with S = diag(rho^-1/2) and L the 5-point Dirichlet
// Laplacian / h^2.  A workgroup of 512 threads (its two LDS stages allow three workgroups per
// CU, so eight waves each keep the CU busy) takes TILE = 256 NPT nodes and CPT columns in two
// stages: z = S x on the tile +-2N, then w = D (L z) on the tile +-N (zero outside the
// grid: the second Laplacian also sees Dirichlet values), then y = a S L w + b x + g Z on the
// tile.  x is read once from HBM for the staging (its tile-interior values again from L2 for
// the b x term); D and rho come from L2 after the first column group.
template <int CPT, int NPT, bool HZ>
__global__ void __launch_bounds__(512) spmm_plate_kernel(
    const OpDev *__restrict__ ops, const double *__restrict__ X, const double *__restrict__ Z,
    double *__restrict__ Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
    const int32_t *__restrict__ lock, const double *__restrict__ coef,
    const int32_t *__restrict__ mdeg, int32_t step, const int32_t *__restrict__ cdeg,
    int32_t mtot) {
  constexpr int TILE = 256 * NPT;
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.z;
  if (mdeg && step >= mdeg[b]) return;
  const OpDev op = ops[b];
  const int N = op.N;
  const int64_t n = op.n;
  const int64_t p0 = (int64_t)blockIdx.x * TILE;
  if (p0 >= n) return;
  int32_t c0, cnt;
  col_range(mode, k, lock, b, c0, cnt);
  const int j0 = blockIdx.y * CPT;
  if (j0 >= cnt) return;
  const int jn = min(CPT, cnt - j0);
  bool act[CPT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    act[j] = j < jn && column_active(cdeg, mtot, step, b, k, c0 + j0 + j);
    any = any || act[j];
  }
  if (!any) return;
  const int span = TILE + 4 * N;                 // z: nodes [p0 - 2N, p0 + TILE + 2N)
  const int wspan = TILE + 2 * N;                // w: nodes [p0 - N, p0 + TILE + N)
  double *sz = reinterpret_cast<double *>(smem_raw);
  double *sw = sz + CPT * span;
  const int tid = threadIdx.x;
  const int64_t off = (int64_t)b * bs + (int64_t)(c0 + j0) * ld;
  const double *xb = X + off;
  const double *D = op.wx, *rho = op.wy;
  const double ih2 = (double)(N + 1) * (double)(N + 1);
  constexpr int U = 4;
  for (int e0 = tid; e0 < span; e0 += 512 * U) {
    double v[U][CPT], sq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 512;
      const int64_t q = p0 - 2 * N + e;
      const bool in = e < span && q >= 0 && q < n;
      sq[u] = in ? rho[q] : 1.0;
#pragma unroll
      for (int j = 0; j < CPT; ++j) v[u][j] = (act[j] && in) ? xb[(int64_t)j * ld + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * 512;
      if (e < span) {
        const double s = 1.0 / sqrt(sq[u]);
#pragma unroll
        for (int j = 0; j < CPT; ++j)
          if (act[j]) sz[j * span + e] = s * v[u][j];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < wspan; e += 512) {
    const int64_t q = p0 - N + e;
    if (q < 0 || q >= n) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) sw[j * wspan + e] = 0.0;
      continue;
    }
    const int qi = (int)q, iy = qi / N, ix = qi - iy * N;
    const double d = D[q] * ih2;
    const int ez = e + N;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (!act[j]) continue;
      const double *zj = sz + j * span;
      double lz = 4.0 * zj[ez];
      if (ix > 0) lz -= zj[ez - 1];
      if (ix < N - 1) lz -= zj[ez + 1];
      if (iy > 0) lz -= zj[ez - N];
      if (iy < N - 1) lz -= zj[ez + N];
      sw[j * wspan + e] = d * lz;
    }
  }
  __syncthreads();
  const double a = coef[3 * b + 0], bc = coef[3 * b + 1], g = coef[3 * b + 2];
#pragma unroll
  for (int t = 0; t < NPT / 2; ++t) {
    const int64_t p = p0 + t * 512 + tid;
    if (p >= n) break;
    const int pi = (int)p, iy = pi / N, ix = pi - iy * N;
    const double sp = ih2 / sqrt(rho[p]);
    const int e = t * 512 + tid + N;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (!act[j]) continue;
      const double *wj = sw + j * wspan;
      double lw = 4.0 * wj[e];
      if (ix > 0) lw -= wj[e - 1];
      if (ix < N - 1) lw -= wj[e + 1];
      if (iy > 0) lw -= wj[e - N];
      if (iy < N - 1) lw -= wj[e + N];
      const int64_t o = off + (int64_t)j * ld + p;
      double r = a * (sp * lw) + bc * X[o];
      if constexpr (HZ) r += g * __builtin_nontemporal_load(&Z[o]);
      __builtin_nontemporal_store(r, &Y[o]);
    }
  }
}

// The plate step with the largest tile <= `tile` whose two LDS stages fit in kStageBytes.
static hipError_t launch_plate(const OpDev *ops, int B, int64_t nmax, int32_t Nmax,
                               const double *X, const double *Z, double *Y, int64_t ld,
                               int64_t bs, int32_t mode, int32_t k, const int32_t *lock,
                               const double *coef, bool has_z, const int32_t *mdeg, int32_t step,
                               int tile, const int32_t *cdeg, int32_t mtot, hipStream_t st);

template <int CPT, typename T, bool SRC>
static bool launch_lds(const OpDev *ops, int B, int32_t kind, bool pot, int64_t nmax, int32_t Nmax,
                       const T *X, const T *Z, T *Y, int64_t ld, int64_t bs, int32_t mode,
                       int32_t k, const int32_t *lock, const double *coef, int hz, const T *R,
                       const double *src, const int32_t *mdeg, int32_t step,
                       const int32_t *cdeg, int32_t mtot, hipStream_t st) {
  constexpr int NPT = 8 / CPT, TILE = 256 * NPT;
  const int64_t H = (kind == SCSF_STENCIL9) ? (int64_t)Nmax + 1 : Nmax;
  const size_t shm = (size_t)CPT * (TILE + 2 * H) * sizeof(T);
  if (shm > kStageBytes) return false;
  dim3 grid((unsigned)ceil_div(nmax, TILE), (unsigned)ceil_div(k, CPT), (unsigned)B);
  auto go = [&](auto kern) {
    kern<<<grid, 256, shm, st>>>(ops, X, Z, Y, ld, bs, mode, k, lock, coef, R, src, mdeg, step,
                                 cdeg, mtot);
  };
  if (kind == SCSF_STENCIL5 && !pot) {
    if (hz) go(spmm_lds_kernel<SCSF_STENCIL5, CPT, NPT, T, SRC, true>);
    else go(spmm_lds_kernel<SCSF_STENCIL5, CPT, NPT, T, SRC, false>);
  } else if (kind == SCSF_STENCIL5) {
    if (hz) go(spmm_lds_kernel<kStencil5V, CPT, NPT, T, SRC, true>);
    else go(spmm_lds_kernel<kStencil5V, CPT, NPT, T, SRC, false>);
  } else {
    if (hz) go(spmm_lds_kernel<SCSF_STENCIL9, CPT, NPT, T, SRC, true>);
    else go(spmm_lds_kernel<SCSF_STENCIL9, CPT, NPT, T, SRC, false>);
  }
  return true;
}

// tile: columns per thread of the LDS-staged step (1, 2, 4 or 8, with 8 / tile nodes per thread),
// the choice the autotuner makes per (n, k).  CSR operators, and grids whose staged rows would
// not fit in 64 KB of LDS, take the register form with 4 columns per thread.
template <typename T, bool SRC>
static hipError_t launch_step(const OpDev *ops, int B, int32_t kind, int64_t nmax,
                              int32_t Nmax, const T *X, const T *Z, T *Y, int64_t ld, int64_t bs,
                              int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                              bool has_z, const T *R, const double *src, const int32_t *mdeg,
                              int32_t step, int tile, bool pot, const int32_t *cdeg,
                              int32_t mtot, hipStream_t st) {
  if (B <= 0 || nmax <= 0 || k <= 0) return hipSuccess;
  if (kind == SCSF_PLATE) {
    if constexpr (std::is_same<T, double>::value && !SRC)
      return launch_plate(ops, B, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef, has_z, mdeg,
                          step, tile, cdeg, mtot, st);
    else
      return hipErrorInvalidValue;                 // the plate family runs in FP64 only
  }
  const int hz = has_z ? 1 : 0;
  bool done = false;
  if (kind != SCSF_CSR && Nmax > 0) {
    if (tile == 1)
      done = launch_lds<1, T, SRC>(ops, B, kind, pot, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   hz, R, src, mdeg, step, cdeg, mtot, st);
    else if (tile == 8)
      done = launch_lds<8, T, SRC>(ops, B, kind, pot, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   hz, R, src, mdeg, step, cdeg, mtot, st);
    else if (tile == 4)
      done = launch_lds<4, T, SRC>(ops, B, kind, pot, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   hz, R, src, mdeg, step, cdeg, mtot, st);
    else
      done = launch_lds<2, T, SRC>(ops, B, kind, pot, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   hz, R, src, mdeg, step, cdeg, mtot, st);
  }
  if (!done)
    launch_reg<4, T, SRC>(ops, B, kind, nmax, X, Z, Y, ld, bs, mode, k, lock, coef, hz, R, src,
                          mdeg, step, cdeg, mtot, st);
  return hipGetLastError();
}

template <int CPT>
static bool plate_fits(int32_t Nmax) {
  constexpr int TILE = 256 * (8 / CPT);
  return (size_t)CPT * (2 * TILE + 6 * (size_t)Nmax) * sizeof(double) <= kStageBytes;
}

template <int CPT>
static void go_plate(const OpDev *ops, int B, int64_t nmax, int32_t Nmax, const double *X,
                     const double *Z, double *Y, int64_t ld, int64_t bs, int32_t mode, int32_t k,
                     const int32_t *lock, const double *coef, bool has_z, const int32_t *mdeg,
                     int32_t step, const int32_t *cdeg, int32_t mtot, hipStream_t st) {
  constexpr int NPT = 8 / CPT, TILE = 256 * NPT;
  const size_t shm = (size_t)CPT * (2 * TILE + 6 * (size_t)Nmax) * sizeof(double);
  dim3 grid((unsigned)ceil_div(nmax, TILE), (unsigned)ceil_div(k, CPT), (unsigned)B);
  if (has_z)
    spmm_plate_kernel<CPT, NPT, true><<<grid, 512, shm, st>>>(ops, X, Z, Y, ld, bs, mode, k, lock,
                                                              coef, mdeg, step, cdeg, mtot);
  else
    spmm_plate_kernel<CPT, NPT, false><<<grid, 512, shm, st>>>(ops, X, Z, Y, ld, bs, mode, k,
                                                               lock, coef, mdeg, step, cdeg, mtot);
}

static hipError_t launch_plate(const OpDev *ops, int B, int64_t nmax, int32_t Nmax,
                               const double *X, const double *Z, double *Y, int64_t ld,
                               int64_t bs, int32_t mode, int32_t k, const int32_t *lock,
                               const double *coef, bool has_z, const int32_t *mdeg, int32_t step,
                               int tile, const int32_t *cdeg, int32_t mtot, hipStream_t st) {
  if (Nmax <= 0) return hipErrorInvalidValue;
  if (tile >= 4 && plate_fits<4>(Nmax))
    go_plate<4>(ops, B, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef, has_z, mdeg, step, cdeg,
                mtot, st);
  else if (tile >= 2 && plate_fits<2>(Nmax))
    go_plate<2>(ops, B, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef, has_z, mdeg, step, cdeg,
                mtot, st);
  else if (plate_fits<1>(Nmax))
    go_plate<1>(ops, B, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef, has_z, mdeg, step, cdeg,
                mtot, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t spmm_step(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                     const double *X, const double *Z, double *Y, int64_t ld, int64_t bs,
                     int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                     bool has_z, hipStream_t st, const int32_t *mdeg, int32_t step, int tile,
                     bool pot, const int32_t *cdeg, int32_t mtot) {
  return launch_step<double, false>(ops, B, kind, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock,
                                    coef, has_z, nullptr, nullptr, mdeg, step, tile, pot, cdeg,
                                    mtot, st);
}

bool spmm_fused_supported(int32_t kind, int32_t Nmax, int S) {
  if (kind != SCSF_STENCIL5 && kind != SCSF_STENCIL9) return false;
  if (Nmax <= 0 || S < 2 || S > 4) return false;
  const int64_t H = (kind == SCSF_STENCIL9) ? (int64_t)Nmax + 1 : Nmax;
  return (size_t)2 * (1024 + 2 * S * H) * sizeof(double) <= kFusedBytes;
}

hipError_t spmm_fused(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                      const double *Xc, const double *Xp, double *Ocur, double *Oprev,
                      int64_t ld, int64_t bs, int32_t mode, int32_t k, const int32_t *lock,
                      const double *coef, int S, hipStream_t st, const int32_t *mdeg,
                      int32_t step0, int tile, bool pot) {
  if (B <= 0 || nmax <= 0 || k <= 0) return hipSuccess;
  if (!spmm_fused_supported(kind, Nmax, S)) return hipErrorInvalidValue;
  bool ok = false;
  if (S == 2)
    ok = launch_fused_s<2>(tile, ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld, bs, mode,
                           k, lock, coef, mdeg, step0, st);
  else if (S == 3)
    ok = launch_fused_s<3>(tile, ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld, bs, mode,
                           k, lock, coef, mdeg, step0, st);
  else
    ok = launch_fused_s<4>(tile, ops, B, kind, pot, nmax, Nmax, Xc, Xp, Ocur, Oprev, ld, bs, mode,
                           k, lock, coef, mdeg, step0, st);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t spmm_step32(const OpDev *ops, int B, int32_t kind, int64_t nmax, int32_t Nmax,
                       const float *X, const float *Z, float *Y, int64_t ld, int64_t bs,
                       int32_t mode, int32_t k, const int32_t *lock, const double *coef,
                       bool has_z, const float *R, const double *src, hipStream_t st,
                       const int32_t *mdeg, int32_t step, int tile, bool pot) {
  if (R)
    return launch_step<float, true>(ops, B, kind, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock,
                                    coef, has_z, R, src, mdeg, step, tile, pot, nullptr, 0, st);
  return launch_step<float, false>(ops, B, kind, nmax, Nmax, X, Z, Y, ld, bs, mode, k, lock, coef,
                                   has_z, nullptr, nullptr, mdeg, step, tile, pot, nullptr, 0,
                                   st);
}

}  // namespace scsf
