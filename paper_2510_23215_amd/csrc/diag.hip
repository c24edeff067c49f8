// Sort diagnostics: how close consecutive operators of an order are, and how much of a
// coefficient field the truncated DFT leaves out (App. F; the appendix on the truncation
// threshold p0).
//
//  highfreq_ratio     : per operator, ||F_high||_F / ||F||_F over its channels, F the 2-D DFT
//                       and high the coefficients whose signed frequency (a in (-p/2, p/2])
//                       reaches p0 on either axis.  ||F||^2 comes from Parseval (p^2 sum f^2);
//                       the low part is transformed directly, one column frequency at a time.
//  subspace_distance  : the one-sided distance ||(I - U U^T) V||_2 between the spans of the
//                       first q columns of two blocks (orthonormal columns): C = U^T V, then
//                       S = R^T R with R = V - U C formed row by row, and the largest
//                       eigenvalue of S by cyclic Jacobi.  Forming R avoids the cancellation
//                       of 1 - sigma_min(C)^2 for nearby subspaces.
#include "common.h"

namespace scsf {

__device__ inline int signed_freq(int a, int p) { return a <= p / 2 ? a : a - p; }

// Block-wide sum of one double per thread (256 threads); every thread gets the result.
__device__ inline double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) highfreq_kernel(const double *__restrict__ fields,
                                                       int32_t channels, int32_t p, int32_t p0,
                                                       double *__restrict__ ratio) {
  extern __shared__ double t[];                   // p complex: one column frequency, all rows
  __shared__ double red[4];
  const int op = blockIdx.x, tid = threadIdx.x;
  double tot = 0.0, low = 0.0;                    // thread partials
  for (int ch = 0; ch < channels; ++ch) {
    const double *f = fields + ((int64_t)op * channels + ch) * (int64_t)p * p;
    for (int64_t e = tid; e < (int64_t)p * p; e += 256) tot += f[e] * f[e];
    for (int a = 0; a < p; ++a) {
      if (abs(signed_freq(a, p)) >= p0) continue;
      // T(y) = sum_x f(y, x) exp(-2 pi i a x / p)
      for (int y = tid; y < p; y += 256) {
        double re = 0.0, im = 0.0;
        for (int x = 0; x < p; ++x) {
          const int m = (int)(((int64_t)a * x) % p);
          double s, c;
          sincospi(2.0 * m / p, &s, &c);
          const double v = f[(int64_t)y * p + x];
          re += v * c;
          im -= v * s;
        }
        t[2 * y] = re;
        t[2 * y + 1] = im;
      }
      __syncthreads();
      // G(b) = sum_y T(y) exp(-2 pi i b y / p) for the low row frequencies b
      for (int b = tid; b < p; b += 256) {
        if (abs(signed_freq(b, p)) >= p0) continue;
        double re = 0.0, im = 0.0;
        for (int y = 0; y < p; ++y) {
          const int m = (int)(((int64_t)b * y) % p);
          double s, c;
          sincospi(2.0 * m / p, &s, &c);
          const double tr = t[2 * y], ti = t[2 * y + 1];
          re += tr * c + ti * s;
          im += ti * c - tr * s;
        }
        low += re * re + im * im;
      }
      __syncthreads();
    }
  }
  const double T = block_sum(tot, red) * (double)p * (double)p;
  const double Lw = block_sum(low, red);
  if (tid == 0) ratio[op] = T > 0.0 ? sqrt(fmax(0.0, (T - Lw) / T)) : 0.0;
}

hipError_t highfreq_ratio(const double *fields, int32_t n_op, int32_t channels, int32_t p,
                          int32_t p0, double *ratio, hipStream_t st) {
  if (n_op <= 0) return hipSuccess;
  highfreq_kernel<<<n_op, 256, (size_t)2 * p * sizeof(double), st>>>(fields, channels, p, p0,
                                                                      ratio);
  return hipGetLastError();
}

constexpr int kDistRows = 64;                     // rows of U and V staged per pass

__global__ void __launch_bounds__(256) subspace_distance_kernel(
    int64_t n, int32_t q, const double *__restrict__ X, int64_t ld, int64_t bs,
    const int32_t *__restrict__ pa, const int32_t *__restrict__ pb, double *__restrict__ out) {
  __shared__ double su[kDistRows * kMaxDistQ], sv[kDistRows * kMaxDistQ];
  __shared__ double C[kMaxDistQ * kMaxDistQ], S[kMaxDistQ * kMaxDistQ];
  const int tid = threadIdx.x;
  const double *U = X + (int64_t)pa[blockIdx.x] * bs, *V = X + (int64_t)pb[blockIdx.x] * bs;
  const int qq = q * q;
  // pass 1: C = U^T V; thread e owns entries e, e + 256, ... (at most 4 for q <= 32)
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = 0; r0 < n; r0 += kDistRows) {
    const int nr = (int)min<int64_t>(kDistRows, n - r0);
    __syncthreads();
    for (int e = tid; e < kDistRows * q; e += 256) {
      const int r = e % kDistRows, c = e / kDistRows;
      su[c * kDistRows + r] = r < nr ? U[(int64_t)c * ld + r0 + r] : 0.0;
      sv[c * kDistRows + r] = r < nr ? V[(int64_t)c * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
      const int e = tid + 256 * s;
      if (e >= qq) break;
      const int i = e / q, j = e % q;
      double a = 0.0;
      for (int r = 0; r < kDistRows; ++r) a += su[i * kDistRows + r] * sv[j * kDistRows + r];
      acc[s] += a;
    }
  }
  for (int s = 0; s < 4; ++s) {
    const int e = tid + 256 * s;
    if (e < qq) C[e] = acc[s];                    // C[i q + j] = u_i . v_j
    acc[s] = 0.0;
  }
  // pass 2: S = R^T R, R = V - U C, staged in sv row chunk by row chunk
  for (int64_t r0 = 0; r0 < n; r0 += kDistRows) {
    const int nr = (int)min<int64_t>(kDistRows, n - r0);
    __syncthreads();
    for (int e = tid; e < kDistRows * q; e += 256) {
      const int r = e % kDistRows, c = e / kDistRows;
      su[c * kDistRows + r] = r < nr ? U[(int64_t)c * ld + r0 + r] : 0.0;
      sv[c * kDistRows + r] = r < nr ? V[(int64_t)c * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    // R[r][j] = V[r][j] - sum_i U[r][i] C[i][j]; each thread finishes whole entries of R
    double rv[8];
    int cnt = 0;
    for (int e = tid; e < kDistRows * q; e += 256) {
      const int r = e % kDistRows, j = e / kDistRows;
      double v = sv[j * kDistRows + r];
      for (int i = 0; i < q; ++i) v -= su[i * kDistRows + r] * C[i * q + j];
      rv[cnt++] = v;
    }
    __syncthreads();
    cnt = 0;
    for (int e = tid; e < kDistRows * q; e += 256) {
      const int r = e % kDistRows, j = e / kDistRows;
      sv[j * kDistRows + r] = rv[cnt++];
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
      const int e = tid + 256 * s;
      if (e >= qq) break;
      const int i = e / q, j = e % q;
      double a = 0.0;
      for (int r = 0; r < kDistRows; ++r) a += sv[i * kDistRows + r] * sv[j * kDistRows + r];
      acc[s] += a;
    }
  }
  for (int s = 0; s < 4; ++s) {
    const int e = tid + 256 * s;
    if (e < qq) S[e] = acc[s];
  }
  __syncthreads();
  // largest eigenvalue of the symmetric S: cyclic Jacobi in one thread
  if (tid == 0) {
    for (int i = 0; i < q; ++i)
      for (int j = i + 1; j < q; ++j) S[j * q + i] = S[i * q + j] = 0.5 * (S[i * q + j] + S[j * q + i]);
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0, dia = 0.0;
      for (int i = 0; i < q; ++i) {
        dia += S[i * q + i] * S[i * q + i];
        for (int j = i + 1; j < q; ++j) off += S[i * q + j] * S[i * q + j];
      }
      if (off <= 1e-32 * dia || off == 0.0) break;
      for (int i = 0; i < q; ++i)
        for (int j = i + 1; j < q; ++j) {
          const double aij = S[i * q + j];
          if (aij == 0.0) continue;
          const double th = (S[j * q + j] - S[i * q + i]) / (2.0 * aij);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
          for (int k = 0; k < q; ++k) {          // columns i, j
            const double ski = S[k * q + i], skj = S[k * q + j];
            S[k * q + i] = c * ski - sn * skj;
            S[k * q + j] = sn * ski + c * skj;
          }
          for (int k = 0; k < q; ++k) {          // rows i, j
            const double sik = S[i * q + k], sjk = S[j * q + k];
            S[i * q + k] = c * sik - sn * sjk;
            S[j * q + k] = sn * sik + c * sjk;
          }
        }
    }
    double lmax = 0.0;
    for (int i = 0; i < q; ++i) lmax = fmax(lmax, S[i * q + i]);
    out[blockIdx.x] = sqrt(lmax);
  }
}

hipError_t subspace_distance(int64_t n, int32_t q, const double *X, int64_t ld, int64_t bs,
                             const int32_t *pa, const int32_t *pb, int32_t P, double *out,
                             hipStream_t st) {
  if (P <= 0) return hipSuccess;
  subspace_distance_kernel<<<P, 256, 0, st>>>(n, q, X, ld, bs, pa, pb, out);
  return hipGetLastError();
}

}  // namespace scsf
