// Truncated-FFT greedy ordering of the operator sequence (Algorithm 2, Section 3.1).
//
//  dft_features   : P_low = the p0 x p0 corner of the 2-D DFT of each parameter field, / p^2.
//                   Only p0 of the p frequencies are needed per axis, so the transform is two
//                   small dense DFT passes (rows, then columns) instead of a full FFT.
//  pair_distances : all squared Frobenius distances between feature blocks (summed over
//                   channels).
//  greedy_order   : the greedy nearest-neighbour walk; the sequential pick runs in one
//                   workgroup with a masked (distance, index) arg-min per step, so exact ties
//                   go to the lowest index.
#include "common.h"

namespace scsf {

__global__ void __launch_bounds__(256) dft_kernel(const double *__restrict__ fields, int32_t p,
                                                  int32_t p0, double *__restrict__ feats) {
  extern __shared__ double f1[];                    // p x p0 complex: row transform
  const int64_t fc = blockIdx.x;                    // (operator, channel)
  const double *P = fields + fc * (int64_t)p * p;
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int e = tid; e < p * p0; e += NT) {
    const int y = e / p0, k2 = e % p0;
    double re = 0.0, im = 0.0;
    for (int x = 0; x < p; ++x) {
      const int m = (int)(((int64_t)k2 * x) % p);
      double s, c;
      sincospi(2.0 * m / p, &s, &c);
      const double v = P[(int64_t)y * p + x];
      re += v * c;
      im -= v * s;
    }
    f1[2 * e] = re;
    f1[2 * e + 1] = im;
  }
  __syncthreads();
  const double scale = 1.0 / ((double)p * p);
  for (int e = tid; e < p0 * p0; e += NT) {
    const int k1 = e / p0, k2 = e % p0;
    double re = 0.0, im = 0.0;
    for (int y = 0; y < p; ++y) {
      const int m = (int)(((int64_t)k1 * y) % p);
      double s, c;
      sincospi(2.0 * m / p, &s, &c);
      const double a = f1[2 * (y * p0 + k2)], bi = f1[2 * (y * p0 + k2) + 1];
      re += a * c + bi * s;                          // (a + i b)(c - i s)
      im += bi * c - a * s;
    }
    double *o = feats + (fc * p0 * p0 + e) * 2;
    o[0] = re * scale;
    o[1] = im * scale;
  }
}

hipError_t dft_features(const double *fields, int32_t n_op, int32_t channels, int32_t p,
                        int32_t p0, double *feats, hipStream_t st) {
  if (n_op <= 0) return hipSuccess;
  const size_t lds = (size_t)p * p0 * 2 * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  dft_kernel<<<(unsigned)((int64_t)n_op * channels), 256, lds, st>>>(fields, p, p0, feats);
  return hipGetLastError();
}

// D[i*n + j] = sum_f |F_i(f) - F_j(f)|^2, 16 x 16 tile of pairs per workgroup
__global__ void __launch_bounds__(256) dist_kernel(const double *__restrict__ F, int32_t n,
                                                   int32_t flen, double *__restrict__ D) {
  constexpr int TC = 32;                             // complex entries staged per pass
  __shared__ double fi[16][2 * TC + 1], fj[16][2 * TC + 1];
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  const int i = blockIdx.y * 16 + ti, j = blockIdx.x * 16 + tj;
  double acc = 0.0;
  for (int f0 = 0; f0 < flen; f0 += TC) {
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 2 * TC; e += 256) {
      const int r = e / (2 * TC), q = e % (2 * TC);
      const int ii = blockIdx.y * 16 + r, jj = blockIdx.x * 16 + r;
      const bool okf = f0 * 2 + q < flen * 2;
      fi[r][q] = (ii < n && okf) ? F[(int64_t)ii * flen * 2 + f0 * 2 + q] : 0.0;
      fj[r][q] = (jj < n && okf) ? F[(int64_t)jj * flen * 2 + f0 * 2 + q] : 0.0;
    }
    __syncthreads();
    const int cnt = min(TC, flen - f0);
    for (int q = 0; q < cnt; ++q) {
      const double dr = fi[ti][2 * q] - fj[tj][2 * q];
      const double di = fi[ti][2 * q + 1] - fj[tj][2 * q + 1];
      acc += dr * dr + di * di;
    }
  }
  if (i < n && j < n) D[(int64_t)i * n + j] = acc;
}

hipError_t pair_distances(const double *feats, int32_t n_op, int32_t flen, double *D,
                          hipStream_t st) {
  if (n_op <= 0) return hipSuccess;
  dim3 grid((unsigned)ceil_div(n_op, 16), (unsigned)ceil_div(n_op, 16));
  dist_kernel<<<grid, 256, 0, st>>>(feats, n_op, flen, D);
  return hipGetLastError();
}

constexpr int kMaxSortOps = 32768;

// order[0..n) = the walk; order[n] = 1 if a distance on the walk's rows was NaN or infinite.
// Such a distance ranks as +infinity, and among equal keys the lowest unvisited index wins, so
// every step picks an unvisited operator whatever the distances hold.
__global__ void __launch_bounds__(1024) greedy_kernel(const double *__restrict__ D, int32_t n,
                                                      int32_t start, int32_t *__restrict__ order) {
  __shared__ unsigned char visited[kMaxSortOps];
  __shared__ double wv[16];
  __shared__ int wi[16];
  __shared__ int s_cur;
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int j = tid; j < n; j += NT) visited[j] = 0;
  if (tid == 0) { s_cur = start; order[0] = start; }
  __syncthreads();
  if (tid == 0) visited[start] = 1;
  int bad = 0;
  for (int step = 1; step < n; ++step) {
    __syncthreads();
    const int cur = s_cur;
    double best = INFINITY;
    int bi = 0x7fffffff;
    for (int j = tid; j < n; j += NT) {
      if (visited[j]) continue;
      double d = D[(int64_t)cur * n + j];
      if (!isfinite(d)) { d = INFINITY; bad = 1; }
      if (d < best || (d == best && j < bi)) { best = d; bi = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_down(best, o, 64);
      const int oi = __shfl_down(bi, o, 64);
      if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if ((tid & 63) == 0) { wv[tid >> 6] = best; wi[tid >> 6] = bi; }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < NT / 64; ++w)
        if (wv[w] < best || (wv[w] == best && wi[w] < bi)) { best = wv[w]; bi = wi[w]; }
      // an unvisited index always exists here (step < n), and every unvisited index is a
      // candidate with a finite or +infinity key, so bi < n
      order[step] = bi;
      visited[bi] = 1;
      s_cur = bi;
    }
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) order[n] = bad ? 1 : 0;
}

hipError_t greedy_order(const double *D, int32_t n_op, int32_t start, int32_t *order,
                        hipStream_t st) {
  if (n_op <= 0) return hipSuccess;
  if (n_op > kMaxSortOps) return hipErrorInvalidValue;
  greedy_kernel<<<1, 1024, 0, st>>>(D, n_op, start, order);
  return hipGetLastError();
}

}  // namespace scsf
