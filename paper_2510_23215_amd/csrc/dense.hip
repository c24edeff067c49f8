// Small dense kernels of one outer iteration, one workgroup per problem:
//   chol_inv   : scaled Cholesky of a Gram matrix and its inverse factor (CholeskyQR, the QR
//                step of Algorithm 3, done as CholeskyQR2 with a shifted fallback);
//   jacobi_eig : eigen-decomposition of the projected matrix (the reduced problem
//                G W = W Theta of Algorithm 3) by parallel cyclic Jacobi.
// Matrices live in LDS when they fit (160 KB per workgroup on gfx950), otherwise in a global
// scratch area that stays resident in L2.
#include "common.h"

namespace scsf {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kLdsDoubles = 19456;                  // 152 KB of matrix storage in LDS
__device__ inline int64_t upk(int i, int j) { return (int64_t)j * (j + 1) / 2 + i; }  // i <= j

// flag bits: 1 = Cholesky breakdown, 2 = NaN/Inf, 4 = shifted factorisation used
//
// Thread layout: 512 threads as 16 (tx) x 32 (ty); loops over packed-triangle elements walk
// rows with tx and columns with ty, so no index needs an integer division.  Each step of the
// factorisation and of the inversion needs a single barrier: the step's trailing update uses
// the not-yet-scaled pivot row divided by the pivot, and the row is scaled one step later,
// when nobody reads it any more.
// CAP: doubles of LDS for the packed factor (a problem whose packed ka(ka+1)/2 exceeds it works
// in global scratch), sized by the launch for its width.
template <int CAP>
__global__ void __launch_bounds__(512) chol_inv_kernel(
    int64_t n, int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ G,
    double *__restrict__ M, int32_t ldm, int32_t *__restrict__ flag,
    const int32_t *__restrict__ gate, int32_t gate_mask, double *__restrict__ gscr) {
  __shared__ double lds[CAP > 0 ? CAP : 1];
  __shared__ double dsc[kMaxK];
  __shared__ double piv[kMaxK];
  __shared__ double colv[kMaxK];
  __shared__ int s_fail;
  __shared__ double s_shift;
  const int b = blockIdx.x;
  if (gate && !(gate[b] & gate_mask)) return;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  if (ka <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int tx = tid & 15, ty = tid >> 4;              // 16 x 32
  // the packed factor of this problem's active width in LDS when it fits, else global scratch
  const bool in_lds = CAP > 0 && (int64_t)ka * (ka + 1) / 2 <= CAP;
  double *S = in_lds ? lds : gscr + (int64_t)b * kMaxK * (kMaxK + 1);
  const double *Gb = G + (int64_t)b * ldm * ldm;
  double *Mb = M + (int64_t)b * ldm * ldm;

  if (tid == 0) { s_fail = 0; s_shift = 0.0; }
  __syncthreads();
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double sh = s_shift;
    for (int j = tid; j < ka; j += NT) {
      const double d = Gb[j + (int64_t)j * ldm] + sh;
      if (!isfinite(d)) atomicOr(&s_fail, 2);
      if (!(d > 0.0)) atomicOr(&s_fail, 1);
      dsc[j] = (d > 0.0) ? sqrt(d) : 1.0;
    }
    __syncthreads();
    for (int c = ty; c < ka; c += 32)
      for (int i = tx; i <= c; i += 16)
        S[upk(i, c)] = (Gb[i + (int64_t)c * ldm] + (i == c ? sh : 0.0)) / (dsc[i] * dsc[c]);
    __syncthreads();
    // right-looking Cholesky of the scaled Gram matrix; S <- R (upper), R^T R = S
    for (int j = 0; j < ka; ++j) {
      const double p = S[upk(j, j)];
      if (j > 0) {                                       // scale the previous pivot row
        const double rp = sqrt(piv[j - 1]);
        for (int c = j + tid; c < ka; c += NT) S[upk(j - 1, c)] /= rp;
        if (tid == 0) S[upk(j - 1, j - 1)] = rp;
      }
      if (tid == 0) {
        double pv = p;
        if (!(pv > 0.0)) { atomicOr(&s_fail, isfinite(pv) ? 1 : 3); pv = 1.0; }
        piv[j] = pv;
      }
      const double pv = (p > 0.0) ? p : 1.0;
      const double inv = 1.0 / pv;
      for (int c = j + 1 + ty; c < ka; c += 32) {
        const double rc = S[upk(j, c)] * inv;
        for (int i = j + 1 + tx; i <= c; i += 16) S[upk(i, c)] -= S[upk(j, i)] * rc;
      }
      __syncthreads();
    }
    if (tid == 0) S[upk(ka - 1, ka - 1)] = sqrt(piv[ka - 1]);
    const int fnow = s_fail;
    __syncthreads();                                     // every thread has read s_fail
    if (attempt == 0 && (fnow & 1) && !(fnow & 2)) {
      // shifted CholeskyQR: s = 11 (n k + k (k+1)) u ||X||_F^2 (Fukaya et al. 2020)
      if (tid == 0) {
        double tr = 0.0;
        for (int j = 0; j < ka; ++j) tr += Gb[j + (int64_t)j * ldm];
        s_shift = 11.0 * ((double)n * ka + (double)ka * (ka + 1)) * 1.1102230246251565e-16 * tr;
        s_fail = 4;
      }
      __syncthreads();
      continue;
    }
    break;
  }
  // S <- R^-1 in place, column by column: with T = R^-1 already on the columns < j,
  // T[0:j, j] = -T[0:j, 0:j] R[0:j, j] / R_jj and T_jj = 1 / R_jj (both read the original
  // column j, which is overwritten only after the barrier).  Four lanes share each row's
  // dot product.
  for (int j = 0; j < ka; ++j) {
    const double tjj = 1.0 / S[upk(j, j)];
    const int g = tid & 3;
    for (int r = tid >> 2; r < j; r += NT >> 2) {
      double acc = 0.0;
      for (int c = r + g; c < j; c += 4) acc += S[upk(r, c)] * S[upk(c, j)];
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (g == 0) colv[r] = acc;
    }
    __syncthreads();
    for (int r = tid; r < j; r += NT) S[upk(r, j)] = -colv[r] * tjj;
    if (tid == 0) S[upk(j, j)] = tjj;
    __syncthreads();
  }
  for (int c = ty; c < ka; c += 32)
    for (int r = tx; r < ka; r += 16)
      Mb[r + (int64_t)c * ldm] = (r <= c) ? S[upk(r, c)] / dsc[r] : 0.0;
  if (tid == 0 && s_fail) atomicOr(&flag[b], s_fail);
}

// Blocked form of the same factorisation for active widths up to 128 (8 blocks of 16 columns),
// one workgroup of 8 waves per problem.  The scaled matrix lives in a square LDS array A
// (R rows, odd column stride R + 1): R in the upper triangle, the strict upper triangle of T = R^-1 stored
// transposed in the lower triangle, T's diagonal in tdg.  Padding columns up to 16 KW are the
// identity, so every block operation is well defined.  Per block column J: wave 0 factors the
// 16 x 16 diagonal block in registers (lane c holds column c), 16-column panels are solved by
// forward substitution, one thread per column, and the trailing upper tiles are updated with
// f64 MFMA; the inverse takes the diagonal blocks (one wave each) and then one block column of
// T at a time, T(:J, J) = -T(:J, :J) R(:J, J) T_JJ, again on MFMA tiles.  About 3 barriers per
// 16 columns instead of 3 per column.
constexpr int kCbMax = 128;

// C(16x16) = sum over kk of X(i, kk) Y(kk, j), the fragments from the accessors; acc in the
// MFMA D layout (lane holds C[lane/16 + 4 v][lane % 16]).
template <class FX, class FY>
__device__ inline v4d cb_tile(v4d acc, int lane, FX fx, FY fy) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = 4 * s + (lane >> 4), ij = lane & 15;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fx(ij, kk), fy(kk, ij), acc, 0, 0, 0);
  }
  return acc;
}

template <int R>
__global__ void __launch_bounds__(512) chol_inv_blocked_kernel(
    int64_t n, int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ G,
    double *__restrict__ M, int32_t ldm, int32_t *__restrict__ flag,
    const int32_t *__restrict__ gate, int32_t gate_mask) {
  constexpr int LS = R + 1;                  // odd column stride: fragment loads spread over banks
  __shared__ double A[R * LS];
  __shared__ double dsc[R];
  __shared__ double tdg[R];
  __shared__ int s_fail;
  __shared__ double s_shift;
  const int b = blockIdx.x;
  if (gate && !(gate[b] & gate_mask)) return;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  if (ka <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int KW = (ka + 15) / 16, Kp = 16 * KW;
  const double *Gb = G + (int64_t)b * ldm * ldm;
  double *Mb = M + (int64_t)b * ldm * ldm;
  if (tid == 0) { s_fail = 0; s_shift = 0.0; }
  __syncthreads();
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double sh = s_shift;
    for (int j = tid; j < ka; j += NT) {
      const double d = Gb[j + (int64_t)j * ldm] + sh;
      if (!isfinite(d)) atomicOr(&s_fail, 2);
      if (!(d > 0.0)) atomicOr(&s_fail, 1);
      dsc[j] = (d > 0.0) ? sqrt(d) : 1.0;
    }
    __syncthreads();
    // scaled upper triangle; identity on the padding
    for (int e = tid; e < Kp * Kp; e += NT) {
      const int i = e % Kp, c = e / Kp;
      if (i > c) { A[i + c * LS] = 0.0; continue; }
      double v;
      if (c < ka) v = (Gb[i + (int64_t)c * ldm] + (i == c ? sh : 0.0)) / (dsc[i] * dsc[c]);
      else v = (i == c) ? 1.0 : 0.0;
      A[i + c * LS] = v;
    }
    __syncthreads();
    for (int J = 0; J < KW; ++J) {
      const int o = 16 * J;
      // (a) the diagonal block by wave 0: lane c < 16 holds column c of the block
      if (wave == 0) {
        double a[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = (lane < 16 && i <= lane) ? A[(o + i) + (o + lane) * LS] : 0.0;
        int fail = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double d = __shfl(a[j], j, 64);
          if (!(d > 0.0)) { fail |= isfinite(d) ? 1 : 3; d = 1.0; }
          const double r = sqrt(d);
          if (lane == j) a[j] = r;
          else if (lane > j) a[j] = a[j] / r;
#pragma unroll
          for (int i = j + 1; i < 16; ++i) {
            const double rji = __shfl(a[j], i, 64);          // R(j, i) from lane i
            if (lane >= i) a[i] -= rji * a[j];
          }
        }
        if (lane < 16) {
#pragma unroll
          for (int i = 0; i < 16; ++i) if (i <= lane) A[(o + i) + (o + lane) * LS] = a[i];
        }
        if (lane == 0 && fail) atomicOr(&s_fail, fail);
      }
      __syncthreads();
      // (b) the panel R(J, c) = R_JJ^-T A(J, c) for the columns right of the block
      for (int c = o + 16 + tid; c < Kp; c += NT) {
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          double v = A[(o + i) + c * LS];
#pragma unroll
          for (int m = 0; m < i; ++m) v -= A[(o + m) + (o + i) * LS] * x[m];
          x[i] = v / A[(o + i) + (o + i) * LS];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) A[(o + i) + c * LS] = x[i];
      }
      __syncthreads();
      // (c) trailing update A(I, L) -= R(J, I)^T R(J, L), J < I <= L, one tile per wave turn
      const int nr = KW - J - 1;
      for (int t = wave; t < nr * (nr + 1) / 2; t += NT / 64) {
        int L = 0;
        while ((L + 1) * (L + 2) / 2 <= t) ++L;
        const int I = t - L * (L + 1) / 2;
        const int oi = 16 * (J + 1 + I), ol = 16 * (J + 1 + L);
        v4d acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = A[(oi + (lane >> 4) + 4 * v) + (ol + (lane & 15)) * LS];
        acc = cb_tile(acc, lane,
                      [&](int i, int kk) { return -A[(o + kk) + (oi + i) * LS]; },
                      [&](int kk, int j) { return A[(o + kk) + (ol + j) * LS]; });
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(oi + (lane >> 4) + 4 * v) + (ol + (lane & 15)) * LS] = acc[v];
      }
      __syncthreads();
    }
    const int fnow = s_fail;
    __syncthreads();                                     // every thread has read s_fail
    if (attempt == 0 && (fnow & 1) && !(fnow & 2)) {
      // shifted CholeskyQR: s = 11 (n k + k (k+1)) u ||X||_F^2 (Fukaya et al. 2020)
      if (tid == 0) {
        double tr = 0.0;
        for (int j = 0; j < ka; ++j) tr += Gb[j + (int64_t)j * ldm];
        s_shift = 11.0 * ((double)n * ka + (double)ka * (ka + 1)) * 1.1102230246251565e-16 * tr;
        s_fail = 4;
      }
      __syncthreads();
      continue;
    }
    break;
  }
  // T = R^-1.  Diagonal blocks first, wave J for block J: lane c < 16 solves column c of
  // T_JJ by back substitution; T_JJ(i, c), i < c, goes to A(o + c, o + i), the diagonal to tdg.
  if (wave < KW) {
    const int o = 16 * wave;
    double t[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double v = 0.0;
      if (lane < 16 && i <= lane) {
        if (i == lane) {
          v = 1.0 / A[(o + i) + (o + i) * LS];
        } else {
#pragma unroll
          for (int m = i + 1; m < 16; ++m)
            if (m <= lane) v -= A[(o + i) + (o + m) * LS] * t[m];
          v /= A[(o + i) + (o + i) * LS];
        }
      }
      t[i] = v;
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i < lane) A[(o + lane) + (o + i) * LS] = t[i];
        else if (i == lane) tdg[o + i] = t[i];
      }
    }
  }
  __syncthreads();
  // T(I, J), I < J, one block column at a time: W_M = R(M, J) T_JJ over R(M, J) (M < J), then
  // T(I, J) = -sum_{M = I}^{J-1} T(I, M) W_M, stored transposed in the lower triangle.
  auto Tel = [&](int r, int c) -> double {             // T(r, c), r <= c
    return (r == c) ? tdg[r] : A[c + r * LS];
  };
  for (int J = 1; J < KW; ++J) {
    const int oj = 16 * J;
    for (int Mi = wave; Mi < J; Mi += NT / 64) {
      const int om = 16 * Mi;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
      acc = cb_tile(acc, lane,
                    [&](int i, int kk) { return A[(om + i) + (oj + kk) * LS]; },
                    [&](int kk, int j) { return kk <= j ? Tel(oj + kk, oj + j) : 0.0; });
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(om + (lane >> 4) + 4 * v) + (oj + (lane & 15)) * LS] = acc[v];
    }
    __syncthreads();
    for (int I = wave; I < J; I += NT / 64) {
      const int oi = 16 * I;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
      for (int Mi = I; Mi < J; ++Mi) {
        const int om = 16 * Mi;
        acc = cb_tile(acc, lane,
                      [&](int i, int kk) {
                        const int r = oi + i, c = om + kk;
                        return r <= c ? -Tel(r, c) : 0.0;
                      },
                      [&](int kk, int j) { return A[(om + kk) + (oj + j) * LS]; });
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(oj + (lane & 15)) + (oi + (lane >> 4) + 4 * v) * LS] = acc[v];
    }
    __syncthreads();
  }
  // M = D^-1/2 T on the active block, zero below the diagonal
  for (int e = tid; e < ka * ka; e += NT) {
    const int r = e % ka, c = e / ka;
    Mb[r + (int64_t)c * ldm] = (r <= c) ? Tel(r, c) / dsc[r] : 0.0;
  }
  if (tid == 0 && s_fail) atomicOr(&flag[b], s_fail);
}

hipError_t chol_inv(int B, int64_t n, int32_t k, const int32_t *lock, const double *G, double *M,
                    int32_t ldm, int32_t *flag, const int32_t *gate, int32_t gate_mask,
                    double *scratch, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  // Both forms size their LDS for the launch's width, so narrow blocks leave room on the CU
  // for other lanes' work.  Blocked form (k <= 128): an R x (R + 1) array, R = k rounded up to
  // 64 / 80 / 96 / 112 / 128.  Packed form (wider): each workgroup keeps its packed R
  // (inverted in place) in LDS when its active width fits the launch's capacity, else in
  // global scratch, so wide blocks move into LDS as their pairs lock.
  const int kr = (int)round_up(k, 16);
  if (kr <= 64)
    chol_inv_blocked_kernel<64><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask);
  else if (kr <= 80)
    chol_inv_blocked_kernel<80><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask);
  else if (kr <= 96)
    chol_inv_blocked_kernel<96><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask);
  else if (kr <= 112)
    chol_inv_blocked_kernel<112><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask);
  else if (k <= kCbMax)
    chol_inv_blocked_kernel<128><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask);
  else if (k <= 160)                     // the packed factor of width 160: 103 KB
    chol_inv_kernel<160 * 161 / 2><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate,
                                                      gate_mask, scratch);
  else
    chol_inv_kernel<kLdsDoubles><<<B, 512, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask,
                                                    scratch);
  return hipGetLastError();
}

// -------------------------------------------------------------------------------- Jacobi
// Parallel cyclic Jacobi in two kernels.
//   jacobi_values : one workgroup per problem keeps the symmetric matrix (upper triangle,
//                   packed) in LDS.  Each round of the round-robin ordering rotates K/2
//                   disjoint index pairs; every 2x2 block (pair a, pair b), a <= b, is read once,
//                   transformed by J_a^T B J_b and written once, so a round touches each stored
//                   entry once.  The rotations are recorded; after every sweep the largest
//                   relative off-diagonal entry is checked directly.
//   jacobi_vectors: the eigenvector matrix Z = product of the recorded rotations, built by
//                   many workgroups at once (each row of Z evolves on its own).
__device__ inline void rr_pair(int r, int s, int K, int &p, int &q) {
  // round-robin tournament: every pair of 0..K-1 meets once in rounds 0..K-2
  if (s == 0) { p = K - 1; q = r; }
  else { p = (r + s) % (K - 1); q = (r - s + (K - 1)) % (K - 1); }
}

__device__ inline int pk(int i, int j) {              // packed upper triangle, any order
  return (i <= j) ? (j * (j + 1) / 2 + i) : (i * (i + 1) / 2 + j);
}

constexpr int kJacobiMaxSweeps = 24;
constexpr double kJacobiTol = 1e-15;                   // smallest relative rotation threshold

int64_t jacobi_record_elems(int32_t k) {
  const int64_t K = k + (k & 1);
  return (int64_t)kJacobiMaxSweeps * (K - 1) * (K / 2) * 2 + (int64_t)kJacobiMaxSweeps * (K - 1);
}

// One workgroup of 1024 threads per problem.  The 2x2-block updates of a round are dealt
// evenly: block e of the packed triangle of pair indices (a <= b) goes to thread e mod 1024, and
// each thread decodes its blocks once before the sweeps.
constexpr int kJacobiThreads = 1024;
constexpr int kJacobiBlocksPerThread =
    ((kMaxK / 2) * (kMaxK / 2 + 1) / 2 + kJacobiThreads - 1) / kJacobiThreads;

// CAP: doubles of LDS for the packed matrix (a problem whose packed K(K+1)/2 exceeds it works in
// global scratch); the launch sizes it for its width, so narrow blocks leave LDS to other work
template <int CAP>
__global__ void __launch_bounds__(kJacobiThreads) jacobi_values_kernel(
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ Gin, int32_t ldm,
    double *__restrict__ theta, int32_t *__restrict__ rank_out, double *__restrict__ rec,
    int64_t rec_stride, int32_t *__restrict__ nsweeps, int32_t *__restrict__ flag,
    double *__restrict__ gscr, double stop) {
  constexpr int NT = kJacobiThreads, MAXE = kJacobiBlocksPerThread;
  __shared__ double lds[CAP > 0 ? CAP : 1];
  __shared__ int2 rpq[kMaxK / 2 + 1];
  __shared__ double2 rcs[kMaxK / 2 + 1];
  __shared__ int s_any[2];
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  const int tid = threadIdx.x;
  if (ka <= 0) { if (tid == 0) nsweeps[b] = 0; return; }
  const int tx = tid & 15, ty = tid >> 4;              // 16 x 64
  const int K = ka + (ka & 1), half = K / 2;
  const bool in_lds = CAP > 0 && (int64_t)K * (K + 1) / 2 <= CAP;
  double *S = in_lds ? lds : gscr + (int64_t)b * kMaxK * (kMaxK + 1);
  const double *Gb = Gin + (int64_t)b * ldm * ldm;
  double *R = rec + (int64_t)b * rec_stride;           // (c, s) per (sweep, round, slot)
  double *Ract = R + (int64_t)kJacobiMaxSweeps * (K - 1) * half * 2;
  for (int c = ty; c < K; c += NT / 16)
    for (int i = tx; i <= c; i += 16)
      S[pk(i, c)] = (i < ka && c < ka) ? Gb[i + (int64_t)c * ldm] : 0.0;  // zero dummy index
  // this thread's 2x2 blocks (aa, bb), aa <= bb < half, as aa | bb << 16 (none: ~0u)
  const int nblk = half * (half + 1) / 2;
  uint32_t blk[MAXE];
#pragma unroll
  for (int u = 0; u < MAXE; ++u) {
    const int e = tid + u * NT;
    uint32_t v = ~0u;
    if (e < nblk) {
      int bb = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (bb * (bb + 1) / 2 > e) --bb;
      while ((bb + 1) * (bb + 2) / 2 <= e) ++bb;
      v = (uint32_t)(e - bb * (bb + 1) / 2) | ((uint32_t)bb << 16);
    }
    blk[u] = v;
  }
  if (tid == 0) { s_any[0] = 0; s_any[1] = 0; }
  __syncthreads();
  // largest relative off-diagonal entry (all threads get the value)
  auto max_off = [&]() {
    double off = 0.0;
    for (int c = ty; c < ka; c += NT / 16)
      for (int i = tx; i < c; i += 16) {
        const double den = sqrt(fabs(S[pk(i, i)] * S[pk(c, c)]));
        const double v = fabs(S[pk(i, c)]);
        off = fmax(off, (v > 1e-300) ? v / fmax(den, 1e-300) : 0.0);
      }
    for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_down(off, o, 64));
    if ((tid & 63) == 0) sh[tid >> 6] = off;
    __syncthreads();
    double m = sh[0];
    for (int w = 1; w < NT / 64; ++w) m = fmax(m, sh[w]);
    __syncthreads();
    return m;
  };
  // entries below a tenth of the stopping level are left alone: the sweep ends at `stop`
  // anyway, and a 2x2 block whose two rotations are both skipped costs no LDS traffic
  const double rthr = fmax(kJacobiTol, 0.1 * stop);
  int sweep = 0;
  bool converged = !(max_off() > stop);              // already diagonal to the requested level
  for (; sweep < kJacobiMaxSweeps && !converged; ++sweep) {
    for (int r = 0; r < K - 1; ++r) {
      // two barriers per round: (A) rotations ready, (B) block updates done.  The flag of
      // the next round is reset before (A), after every thread read it before (B) last round.
      const int par = r & 1;
      for (int a = tid; a < half; a += NT) {
        int p, q;
        rr_pair(r, a, K, p, q);
        double c = 1.0, sn = 0.0;
        const double gpp = S[pk(p, p)], gqq = S[pk(q, q)], gpq = S[pk(p, q)];
        if (fabs(gpq) > rthr * sqrt(fabs(gpp * gqq)) && fabs(gpq) > 1e-300) {
          const double tau = (gqq - gpp) / (2.0 * gpq);
          double t;
          if (fabs(tau) > 1e150) t = 0.5 / tau;
          else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = c * t;
          s_any[par] = 1;
        }
        rpq[a] = make_int2(p, q);
        rcs[a] = make_double2(c, sn);
        double *o = R + (((int64_t)sweep * (K - 1) + r) * half + a) * 2;
        o[0] = c;
        o[1] = sn;
      }
      if (tid == 0) s_any[par ^ 1] = 0;
      __syncthreads();                                   // (A)
      const int any = s_any[par];
      if (tid == 0) Ract[(int64_t)sweep * (K - 1) + r] = any ? 1.0 : 0.0;
      if (any) {
#pragma unroll
        for (int u = 0; u < MAXE; ++u) {
          if (blk[u] == ~0u) continue;
          const int aa = (int)(blk[u] & 0xffffu), bb = (int)(blk[u] >> 16);
          const double2 ra = rcs[aa], rb = rcs[bb];
          const double ca = ra.x, sa = ra.y, cb = rb.x, sb = rb.y;
          if (sa == 0.0 && sb == 0.0) continue;
          const int2 qa = rpq[aa];
          const int pa = qa.x, qaa = qa.y;
          if (aa == bb) {                                // the pair's own 2x2 block
            const int ipp = pk(pa, pa), iqq = pk(qaa, qaa), ipq = pk(pa, qaa);
            const double gpp = S[ipp], gqq = S[iqq], gpq = S[ipq];
            const double t = sa / ca;
            S[ipp] = gpp - t * gpq;
            S[iqq] = gqq + t * gpq;
            S[ipq] = 0.0;
          } else {
            const int2 qb = rpq[bb];
            const int pb = qb.x, qbb = qb.y;
            const int i11 = pk(pa, pb), i12 = pk(pa, qbb), i21 = pk(qaa, pb), i22 = pk(qaa, qbb);
            const double g11 = S[i11], g12 = S[i12], g21 = S[i21], g22 = S[i22];
            const double r11 = ca * g11 - sa * g21, r12 = ca * g12 - sa * g22;
            const double r21 = sa * g11 + ca * g21, r22 = sa * g12 + ca * g22;
            S[i11] = cb * r11 - sb * r12;
            S[i12] = sb * r11 + cb * r12;
            S[i21] = cb * r21 - sb * r22;
            S[i22] = sb * r21 + cb * r22;
          }
        }
      }
      __syncthreads();                                   // (B)
    }
    if (!(max_off() > stop)) {
      converged = true;
      ++sweep;
      break;
    }
  }
  if (tid == 0) {
    nsweeps[b] = sweep;
    if (!converged) atomicOr(&flag[b], 8);
  }
  // ascending order: rank_j = #{i : theta_i < theta_j or (== and i < j)}
  for (int j = tid; j < ka; j += NT) {
    const double tj = S[pk(j, j)];
    int rk = 0;
    for (int i = 0; i < ka; ++i) {
      const double ti = S[pk(i, i)];
      rk += (ti < tj) || (ti == tj && i < j);
    }
    rank_out[(int64_t)b * ldm + j] = rk;
    theta[(int64_t)b * k + l + rk] = tj;
    if (!isfinite(tj)) atomicOr(&flag[b], 2);
  }
}

// grid (ceil(kmax / 8), 1, B): 8 rows of Z per workgroup, 64 slots per row (one per lane).
__global__ void __launch_bounds__(512) jacobi_vectors_kernel(
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ rec, int64_t rec_stride,
    const int32_t *__restrict__ nsweeps, const int32_t *__restrict__ rank_in,
    double *__restrict__ Zout, int32_t ldm) {
  constexpr int RW = 8, CH = 8;                        // rows per workgroup, rounds per stage
  __shared__ double z[RW][kMaxK + 1];
  __shared__ double cs[CH][kMaxK / 2][2];
  __shared__ double act[CH];
  const int b = blockIdx.z;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  const int row0 = blockIdx.x * RW;
  if (ka <= 0 || row0 >= ka) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;             // row w of this block, slot lane(+64)
  const int K = ka + (ka & 1), half = K / 2;
  const int rounds = nsweeps[b] * (K - 1);
  const double *R = rec + (int64_t)b * rec_stride;
  const double *Ract = R + (int64_t)kJacobiMaxSweeps * (K - 1) * half * 2;
  for (int e = tid; e < RW * K; e += 512) {
    const int rr = e / K, j = e % K;
    z[rr][j] = (row0 + rr == j) ? 1.0 : 0.0;
  }
  const int gi = row0 + w;                             // global row of this thread's z row
  for (int g0 = 0; g0 < rounds; g0 += CH) {
    const int nr = min(CH, rounds - g0);
    __syncthreads();
    for (int e = tid; e < nr * half * 2; e += 512) {
      const int rr = e / (half * 2), q = e % (half * 2);
      cs[rr][q >> 1][q & 1] = R[((int64_t)(g0 + rr) * half) * 2 + q];
    }
    if (tid < nr) act[tid] = Ract[g0 + tid];
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      if (act[rr] != 0.0 && gi < ka) {
        const int r = (g0 + rr) % (K - 1);
        for (int a = lane; a < half; a += 64) {
          const double c = cs[rr][a][0], sn = cs[rr][a][1];
          if (sn == 0.0) continue;
          int p, q;
          rr_pair(r, a, K, p, q);
          const double zp = z[w][p], zq = z[w][q];
          z[w][p] = c * zp - sn * zq;
          z[w][q] = sn * zp + c * zq;
        }
      }
      // rotations of one round touch disjoint columns of a row; the wave owning the row is
      // the only writer, so the next round only needs the wave's own ordering
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  if (gi < ka) {
    double *Zb = Zout + (int64_t)b * ldm * ldm;
    const int32_t *rk = rank_in + (int64_t)b * ldm;
    for (int j = lane; j < ka; j += 64) Zb[gi + (int64_t)rk[j] * ldm] = z[w][j];
  }
}

hipError_t jacobi_eig(int B, int32_t k, const int32_t *lock, double *G, double *Z, int32_t ldm,
                      double *theta, int32_t *flag, double *scratch, double *rec,
                      int32_t *ranks, int32_t *nsweeps, hipStream_t st, double stop) {
  if (B <= 0) return hipSuccess;
  const int64_t rs = jacobi_record_elems(k);
  // per problem: the packed matrix in LDS when its active width fits, else global scratch; the
  // LDS array is sized for the launch's width (K = k rounded up to even)
  const int64_t K = k + (k & 1), need = K * (K + 1) / 2;
  if (need <= 64 * 65 / 2)
    jacobi_values_kernel<64 * 65 / 2><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  else if (need <= 80 * 81 / 2)
    jacobi_values_kernel<80 * 81 / 2><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  else if (need <= 96 * 97 / 2)
    jacobi_values_kernel<96 * 97 / 2><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  else if (need <= 128 * 129 / 2)
    jacobi_values_kernel<128 * 129 / 2><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  else if (need <= 160 * 161 / 2)
    jacobi_values_kernel<160 * 161 / 2><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  else
    jacobi_values_kernel<kLdsDoubles><<<B, kJacobiThreads, 0, st>>>(
        k, lock, G, ldm, theta, ranks, rec, rs, nsweeps, flag, scratch, stop);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  jacobi_vectors_kernel<<<dim3((unsigned)ceil_div(k, 8), 1, B), 512, 0, st>>>(
      k, lock, rec, rs, nsweeps, ranks, Z, ldm);
  return hipGetLastError();
}

}  // namespace scsf
