// Small dense kernels of one outer iteration, one workgroup per problem:
//   chol_inv   : scaled Cholesky of a Gram matrix and its inverse factor (CholeskyQR, the QR
//                step of Algorithm 3, done as CholeskyQR2 with a shifted fallback);
//   jacobi_eig : eigen-decomposition of the projected matrix (the reduced problem
//                G W = W Theta of Algorithm 3) by parallel cyclic Jacobi.
// Matrices live in LDS when they fit (160 KB per workgroup on gfx950), otherwise in a global
// scratch area that stays resident in L2.
#include "common.h"

namespace scsf {

constexpr int kLdsDoubles = 19456;                  // 152 KB of matrix storage in LDS
__device__ inline int64_t upk(int i, int j) { return (int64_t)j * (j + 1) / 2 + i; }  // i <= j

// flag bits: 1 = Cholesky breakdown, 2 = NaN/Inf, 4 = shifted factorisation used
template <bool LDS>
__global__ void __launch_bounds__(256) chol_inv_kernel(
    int64_t n, int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ G,
    double *__restrict__ M, int32_t ldm, int32_t *__restrict__ flag,
    const int32_t *__restrict__ gate, int32_t gate_mask, double *__restrict__ gscr) {
  __shared__ double lds[LDS ? kLdsDoubles : 1];
  __shared__ double dsc[kMaxK];
  __shared__ int s_fail;
  __shared__ double s_shift;
  const int b = blockIdx.x;
  if (gate && !(gate[b] & gate_mask)) return;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  if (ka <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  double *S = LDS ? lds : gscr + (int64_t)b * kMaxK * (kMaxK + 1);
  double *T = S + (int64_t)ka * (ka + 1) / 2;
  const double *Gb = G + (int64_t)b * ldm * ldm;
  double *Mb = M + (int64_t)b * ldm * ldm;

  if (tid == 0) { s_fail = 0; s_shift = 0.0; }
  __syncthreads();
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double sh = s_shift;
    for (int j = tid; j < ka; j += NT) {
      const double d = Gb[j + (int64_t)j * ldm] + sh;
      if (!isfinite(d)) atomicOr(&s_fail, 2);
      dsc[j] = (d > 0.0) ? sqrt(d) : 1.0;
      if (!(d > 0.0)) atomicOr(&s_fail, 1);
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)ka * ka; e += NT) {
      const int i = (int)(e % ka), j = (int)(e / ka);
      if (i <= j) S[upk(i, j)] = (Gb[i + (int64_t)j * ldm] + (i == j ? sh : 0.0)) / (dsc[i] * dsc[j]);
    }
    __syncthreads();
    // right-looking Cholesky, S <- R (upper), R^T R = scaled Gram
    for (int j = 0; j < ka; ++j) {
      if (tid == 0) {
        const double piv = S[upk(j, j)];
        if (!(piv > 0.0)) { atomicOr(&s_fail, isfinite(piv) ? 1 : 3); S[upk(j, j)] = 1.0; }
        else S[upk(j, j)] = sqrt(piv);
      }
      __syncthreads();
      const double rjj = S[upk(j, j)];
      for (int c = j + 1 + tid; c < ka; c += NT) S[upk(j, c)] /= rjj;
      __syncthreads();
      const int m = ka - j - 1;
      for (int64_t e = tid; e < (int64_t)m * m; e += NT) {
        const int i = j + 1 + (int)(e % m), c = j + 1 + (int)(e / m);
        if (i <= c) S[upk(i, c)] -= S[upk(j, i)] * S[upk(j, c)];
      }
      __syncthreads();
    }
    if (attempt == 0 && (s_fail & 1) && !(s_fail & 2)) {
      // shifted CholeskyQR: s = 11 (n k + k (k+1)) u ||X||_F^2 (Fukaya et al. 2020)
      __syncthreads();
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
  // T <- R^-1 (upper), column sweep from the last row up
  const int64_t npk2 = (int64_t)ka * (ka + 1) / 2;
  for (int64_t e = tid; e < npk2; e += NT) T[e] = 0.0;
  __syncthreads();
  for (int j = tid; j < ka; j += NT) T[upk(j, j)] = 1.0;
  for (int i = ka - 1; i >= 0; --i) {
    __syncthreads();
    const double rii = S[upk(i, i)];
    for (int c = i + tid; c < ka; c += NT) T[upk(i, c)] /= rii;
    __syncthreads();
    if (i > 0) {
      const int w = ka - i;
      for (int64_t e = tid; e < (int64_t)i * w; e += NT) {
        const int r = (int)(e % i), c = i + (int)(e / i);
        T[upk(r, c)] -= S[upk(r, i)] * T[upk(i, c)];
      }
    }
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)ka * ka; e += NT) {
    const int r = (int)(e % ka), c = (int)(e / ka);
    Mb[r + (int64_t)c * ldm] = (r <= c) ? T[upk(r, c)] / dsc[r] : 0.0;
  }
  if (tid == 0 && s_fail) atomicOr(&flag[b], s_fail);
}

hipError_t chol_inv(int B, int64_t n, int32_t k, const int32_t *lock, const double *G, double *M,
                    int32_t ldm, int32_t *flag, const int32_t *gate, int32_t gate_mask,
                    double *scratch, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  // the packed R and R^-1 fit in LDS for every ka when k(k+1) <= kLdsDoubles
  if ((int64_t)k * (k + 1) <= kLdsDoubles)
    chol_inv_kernel<true><<<B, 256, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask, scratch);
  else
    chol_inv_kernel<false><<<B, 256, 0, st>>>(n, k, lock, G, M, ldm, flag, gate, gate_mask,
                                              scratch);
  return hipGetLastError();
}

// -------------------------------------------------------------------------------- Jacobi
__device__ inline void rr_pair(int r, int s, int K, int &p, int &q) {
  // round-robin tournament: every pair of 0..K-1 meets once in rounds 0..K-2
  if (s == 0) { p = K - 1; q = r; }
  else { p = (r + s) % (K - 1); q = (r - s + (K - 1)) % (K - 1); }
}

template <bool G_LDS, bool Z_LDS>
__global__ void __launch_bounds__(512) jacobi_kernel(
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ Gin,
    double *__restrict__ Zout, int32_t ldm, double *__restrict__ theta, int32_t *__restrict__ flag,
    double *__restrict__ gscr) {
  __shared__ double lds[(G_LDS || Z_LDS) ? kLdsDoubles : 1];
  __shared__ int rp[kMaxK / 2 + 1], rq[kMaxK / 2 + 1], ract[kMaxK / 2 + 1];
  __shared__ double rc[kMaxK / 2 + 1], rs[kMaxK / 2 + 1];
  __shared__ int s_nrot;
  __shared__ int rank[kMaxK];
  const int b = blockIdx.x;
  const int32_t l = lock ? lock[b] : 0;
  const int ka = k - l;
  if (ka <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int sg = ka | 1;                               // odd stride against bank conflicts
  double *Gs = G_LDS ? lds : gscr + (int64_t)b * 2 * kMaxK * (kMaxK + 1);
  double *Zs = Z_LDS ? (G_LDS ? lds + (int64_t)ka * sg : lds)
                     : gscr + (int64_t)b * 2 * kMaxK * (kMaxK + 1) + (int64_t)kMaxK * (kMaxK + 1);
  const double *Gb = Gin + (int64_t)b * ldm * ldm;
#define GG(i, j) Gs[(i) + (int64_t)(j) * sg]
#define ZZ(i, j) Zs[(i) + (int64_t)(j) * sg]
  for (int64_t e = tid; e < (int64_t)ka * ka; e += NT) {
    const int i = (int)(e % ka), j = (int)(e / ka);
    GG(i, j) = Gb[i + (int64_t)j * ldm];
    ZZ(i, j) = (i == j) ? 1.0 : 0.0;
  }
  const int K = ka + (ka & 1);
  const int half = K / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();                                  // every thread has read s_nrot
    if (tid == 0) s_nrot = 0;
    for (int r = 0; r < K - 1; ++r) {
      __syncthreads();
      for (int s = tid; s < half; s += NT) {
        int p, q;
        rr_pair(r, s, K, p, q);
        int act = 0;
        double c = 1.0, sn = 0.0;
        if (p < ka && q < ka) {
          const double gpp = GG(p, p), gqq = GG(q, q), gpq = GG(p, q);
          if (fabs(gpq) > 1e-15 * sqrt(fabs(gpp * gqq)) && fabs(gpq) > 1e-300) {
            const double tau = (gqq - gpp) / (2.0 * gpq);
            double t;
            if (fabs(tau) > 1e150) t = 0.5 / tau;
            else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = c * t;
            act = 1;
          }
        }
        rp[s] = p; rq[s] = q; rc[s] = c; rs[s] = sn; ract[s] = act;
        if (act) atomicAdd(&s_nrot, 1);
      }
      __syncthreads();
      // rows p, q of J^T G
      for (int64_t e = tid; e < (int64_t)half * ka; e += NT) {
        const int s = (int)(e / ka), j = (int)(e % ka);
        if (!ract[s]) continue;
        const int p = rp[s], q = rq[s];
        const double c = rc[s], sn = rs[s];
        const double gp = GG(p, j), gq = GG(q, j);
        GG(p, j) = c * gp - sn * gq;
        GG(q, j) = sn * gp + c * gq;
      }
      __syncthreads();
      // columns p, q of (J^T G) J and of Z J
      for (int64_t e = tid; e < (int64_t)half * ka; e += NT) {
        const int s = (int)(e / ka), i = (int)(e % ka);
        if (!ract[s]) continue;
        const int p = rp[s], q = rq[s];
        const double c = rc[s], sn = rs[s];
        const double gp = GG(i, p), gq = GG(i, q);
        GG(i, p) = c * gp - sn * gq;
        GG(i, q) = sn * gp + c * gq;
        const double zp = ZZ(i, p), zq = ZZ(i, q);
        ZZ(i, p) = c * zp - sn * zq;
        ZZ(i, q) = sn * zp + c * zq;
      }
      __syncthreads();
      for (int s = tid; s < half; s += NT)
        if (ract[s]) { GG(rp[s], rq[s]) = 0.0; GG(rq[s], rp[s]) = 0.0; }
    }
    __syncthreads();
    const int nrot = s_nrot;
    if (nrot == 0) break;
  }
  __syncthreads();
  // ascending order: rank_j = #{i : theta_i < theta_j or (== and i < j)}
  for (int j = tid; j < ka; j += NT) {
    const double tj = GG(j, j);
    int rk = 0;
    for (int i = 0; i < ka; ++i) {
      const double ti = GG(i, i);
      rk += (ti < tj) || (ti == tj && i < j);
    }
    rank[j] = rk;
    theta[(int64_t)b * k + l + rk] = tj;
    if (!isfinite(tj)) atomicOr(&flag[b], 2);
  }
  __syncthreads();
  double *Zb = Zout + (int64_t)b * ldm * ldm;
  for (int64_t e = tid; e < (int64_t)ka * ka; e += NT) {
    const int i = (int)(e % ka), j = (int)(e / ka);
    Zb[i + (int64_t)rank[j] * ldm] = ZZ(i, j);
  }
#undef GG
#undef ZZ
}

hipError_t jacobi_eig(int B, int32_t k, const int32_t *lock, double *G, double *Z, int32_t ldm,
                      double *theta, int32_t *flag, double *scratch, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const int sg = k | 1;
  if ((int64_t)2 * k * sg <= kLdsDoubles)
    jacobi_kernel<true, true><<<B, 512, 0, st>>>(k, lock, G, Z, ldm, theta, flag, scratch);
  else if ((int64_t)k * sg <= kLdsDoubles)
    jacobi_kernel<true, false><<<B, 512, 0, st>>>(k, lock, G, Z, ldm, theta, flag, scratch);
  else
    jacobi_kernel<false, false><<<B, 512, 0, st>>>(k, lock, G, Z, ldm, theta, flag, scratch);
  return hipGetLastError();
}

}  // namespace scsf
