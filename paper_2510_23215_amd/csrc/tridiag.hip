// Symmetric eigen-decomposition of the small projected matrices (the reduced problem
// G W = W Theta of Algorithm 3) without sweeps:
//   tridiag_eig_kernel  : one workgroup per problem.  Householder reduction of the packed
//                         active block to tridiagonal form in LDS; eigenvalues by Sturm
//                         bisection (ascending by construction, several threads per
//                         eigenvalue); eigenvectors of the tridiagonal matrix by inverse
//                         iteration with partial pivoting, re-orthogonalised inside clusters.
//   tridiag_back_kernel : many workgroups.  Eigenvectors of G = the reflectors applied to the
//                         tridiagonal eigenvectors, one wavefront per eigenvector.
// The reduction reads and writes the packed matrix about once per column (2/3 k^3 element
// accesses in all), where a Jacobi sweep touches every element (k - 1) times.
#include "common.h"

namespace scsf {

namespace {

// packed matrix storage in LDS: with the five k-vectors below, 163456 of the 163840 bytes
constexpr int kTriLds = 19136;
constexpr int kInvIters = 3;                       // inverse-iteration passes

__device__ inline int64_t tpk(int i, int j) {     // packed upper triangle, any order
  return (i <= j) ? ((int64_t)j * (j + 1) / 2 + i) : ((int64_t)i * (i + 1) / 2 + j);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Start vector of inverse iteration: a fixed pseudo-random entry in [-1, 1] per (vector, row)
// (distinct start vectors separate the members of a cluster).
__device__ inline double start_entry(int t, int i) {
  uint64_t z = (uint64_t)(t + 1) * 0x9E3779B97F4A7C15ULL + (uint64_t)(i + 1) * 0xBF58476D1CE4E5B9ULL;
  z ^= z >> 31;
  z *= 0x94D049BB133111EBULL;
  z ^= z >> 29;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace

// Per-problem work area: reflectors (k x k), tau (k), LU factors u, v1, v2 and the vectors
// (4 x k x k, entry (i, t) at i * k + t so that the threads of one row are contiguous).
int64_t tridiag_work_elems(int32_t k) { return 5 * (int64_t)k * k + (int64_t)k; }

template <bool LDS>
__global__ void __launch_bounds__(512) tridiag_eig_kernel(
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ Gin, int32_t ldm,
    double *__restrict__ theta, int32_t *__restrict__ flag, double *__restrict__ gscr,
    double *__restrict__ work, int64_t wstride) {
  __shared__ double lds[LDS ? kTriLds : 1];
  __shared__ double dd[kMaxK], ee[kMaxK], e2[kMaxK], pp[kMaxK], lam[kMaxK];
  __shared__ double red[8], red2[8];
  const int b = blockIdx.x;
  const int l = lock ? lock[b] : 0;
  const int ka = k - l;
  if (ka <= 0) return;
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, NW = NT >> 6;
  const int tx = tid & 15, ty = tid >> 4;            // 16 x 32
  const bool in_lds = LDS && (int64_t)ka * (ka + 1) / 2 <= kTriLds;
  double *S = in_lds ? lds : gscr + (int64_t)b * kMaxK * (kMaxK + 1);
  const double *Gb = Gin + (int64_t)b * ldm * ldm;
  double *Wk = work + (int64_t)b * wstride;
  double *refl = Wk, *tau = Wk + (int64_t)k * k;
  double *fu = tau + k, *fv1 = fu + (int64_t)k * k, *fv2 = fv1 + (int64_t)k * k;
  double *fb = fv2 + (int64_t)k * k;

  for (int c = ty; c < ka; c += 32)
    for (int i = tx; i <= c; i += 16) S[tpk(i, c)] = Gb[i + (int64_t)c * ldm];
  __syncthreads();

  // ---- Householder reduction: step j annihilates row j beyond the superdiagonal.
  //      v = x - alpha e_1 (x = row j right of the diagonal, alpha = -sign(x_0) ||x||),
  //      p = tau A22 v, w = p - (tau/2)(v^T p) v, A22 <- A22 - v w^T - w v^T.
  for (int j = 0; j + 2 < ka; ++j) {
    double part = 0.0;
    for (int c = j + 2 + tid; c < ka; c += NT) {
      const double x = S[tpk(j, c)];
      part += x * x;
    }
    part = wave_sum(part);
    if (lane == 0) red[wv] = part;
    __syncthreads();
    double sig = 0.0;
    for (int w = 0; w < NW; ++w) sig += red[w];
    const double x0 = S[tpk(j, j + 1)];
    double v0 = 0.0, t = 0.0, alpha = x0;
    if (sig > 0.0) {
      const double mu = sqrt(x0 * x0 + sig);
      alpha = (x0 > 0.0) ? -mu : mu;
      v0 = x0 - alpha;                                 // same sign as x0: no cancellation
      t = 2.0 / (v0 * v0 + sig);
    }
    if (tid == 0) {
      dd[j] = S[tpk(j, j)];
      ee[j] = alpha;
      tau[j] = t;
    }
    if (t != 0.0) {                                    // the same decision in every thread
      const int g = tid & 3;
      double vp = 0.0;
      for (int i = j + 1 + (tid >> 2); i < ka; i += NT >> 2) {
        double acc = 0.0;
        for (int c = j + 1 + g; c < ka; c += 4) {
          const double vc = (c == j + 1) ? v0 : S[tpk(j, c)];
          acc += S[tpk(i, c)] * vc;
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (g == 0) {
          const double pi = t * acc;
          pp[i] = pi;
          vp += ((i == j + 1) ? v0 : S[tpk(j, i)]) * pi;
        }
      }
      vp = wave_sum(vp);
      if (lane == 0) red2[wv] = vp;
      __syncthreads();                                 // pp and red2 complete; x0 read by all
      double vtp = 0.0;
      for (int w = 0; w < NW; ++w) vtp += red2[w];
      const double K = 0.5 * t * vtp;
      for (int c = j + 1 + ty; c < ka; c += 32) {
        const double vc = (c == j + 1) ? v0 : S[tpk(j, c)];
        const double wc = pp[c] - K * vc;
        for (int i = j + 1 + tx; i <= c; i += 16) {
          const double vi = (i == j + 1) ? v0 : S[tpk(j, i)];
          S[tpk(i, c)] -= vi * wc + (pp[i] - K * vi) * vc;
        }
      }
      if (tid == 0) S[tpk(j, j + 1)] = v0;             // row j now holds the reflector
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (ka >= 2) {
      dd[ka - 2] = S[tpk(ka - 2, ka - 2)];
      ee[ka - 2] = S[tpk(ka - 2, ka - 1)];
    }
    dd[ka - 1] = S[tpk(ka - 1, ka - 1)];
  }
  for (int j = ty; j + 2 < ka; j += 32)
    for (int c = j + 1 + tx; c < ka; c += 16) refl[(int64_t)j * k + c] = S[tpk(j, c)];
  __syncthreads();
  for (int i = tid; i + 1 < ka; i += NT) e2[i] = ee[i] * ee[i];
  __syncthreads();

  // ---- eigenvalues: Sturm-count multisection, G threads per eigenvalue (G + 1 subintervals
  //      per pass).  count(x) = #{eigenvalues < x} from the signs of the LDL^T pivots.
  double gl = 1e300, gu = -1e300, emax2 = 0.0, tnorm1 = 0.0;
  for (int i = 0; i < ka; ++i) {
    const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < ka ? fabs(ee[i]) : 0.0);
    gl = fmin(gl, dd[i] - r);
    gu = fmax(gu, dd[i] + r);
    tnorm1 = fmax(tnorm1, fabs(dd[i]) + r);
    if (i + 1 < ka) emax2 = fmax(emax2, e2[i]);
  }
  const double eps = 1.1102230246251565e-16;
  const double pivmin = 1e-290 * fmax(1.0, emax2);
  {
    const int G = ka <= 64 ? 8 : ka <= 128 ? 4 : 2;
    const int tt = tid / G, g = tid % G, base = lane - g;
    const int te = min(tt, ka - 1);                    // spare threads shadow the last value
    double lo = gl - 4.0 * eps * tnorm1 * ka - pivmin;
    double hi = gu + 4.0 * eps * tnorm1 * ka + pivmin;
    if (tt < (NT / G)) {
      for (int it = 0; it < 200; ++it) {
        if (!(hi - lo > 2.0 * eps * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin)) break;
        const double x = lo + (hi - lo) * (double)(g + 1) / (double)(G + 1);
        double q = dd[0] - x;
        if (fabs(q) <= pivmin) q = -pivmin;
        int cnt = q < 0.0;
        for (int i = 1; i < ka; ++i) {
          q = dd[i] - x - e2[i - 1] / q;
          if (fabs(q) <= pivmin) q = -pivmin;
          cnt += q < 0.0;
        }
        double nlo = lo, nhi = hi;
        for (int s = 0; s < G; ++s) {
          const double xs = __shfl(x, base + s, 64);
          const int cs = __shfl(cnt, base + s, 64);
          if (cs > te) nhi = fmin(nhi, xs);
          else nlo = fmax(nlo, xs);
        }
        if (!(nlo > lo || nhi < hi)) break;            // no progress at this precision
        lo = nlo;
        hi = nhi;
      }
      if (g == 0 && tt < ka) lam[tt] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();
  for (int t = tid; t < ka; t += NT) {
    theta[(int64_t)b * k + l + t] = lam[t];
    if (!isfinite(lam[t])) atomicOr(&flag[b], 2);
  }

  // ---- eigenvectors of the tridiagonal matrix: inverse iteration (T - x I) y = b with
  //      partial pivoting; clusters (gaps <= 1e-3 ||T||_1) get distinct shifts and are
  //      re-orthogonalised (modified Gram-Schmidt, in eigenvalue order) after every pass.
  const double ortol = 1e-3 * tnorm1;
  const double pert = 10.0 * eps * fmax(tnorm1, 1e-300);
  for (int pass = 0; pass < kInvIters; ++pass) {
    for (int t = tid; t < ka; t += NT) {
      int lead = t;
      while (lead > 0 && lam[lead] - lam[lead - 1] <= ortol) --lead;
      const double x = lam[t] + (double)(t - lead) * pert;
      auto rhs = [&](int i) { return pass == 0 ? start_entry(t, i) : fb[(int64_t)i * k + t]; };
      double cd = dd[0] - x, cs = ka > 1 ? ee[0] : 0.0, bc = rhs(0);
      for (int i = 0; i + 1 < ka; ++i) {
        const double sub = ee[i], dn = dd[i + 1] - x, sn = (i + 2 < ka) ? ee[i + 1] : 0.0;
        const double bn = rhs(i + 1);
        double u, v1, v2, bi;
        if (fabs(cd) >= fabs(sub)) {
          const double m = (cd != 0.0) ? sub / cd : 0.0;
          u = cd; v1 = cs; v2 = 0.0; bi = bc;
          cd = dn - m * cs;
          cs = sn;
          bc = bn - m * bc;
        } else {
          const double m = cd / sub;
          u = sub; v1 = dn; v2 = sn; bi = bn;
          cd = cs - m * dn;
          cs = -m * sn;
          bc = bc - m * bn;
        }
        if (fabs(u) < pert) u = (u < 0.0) ? -pert : pert;
        const int64_t o = (int64_t)i * k + t;
        fu[o] = u;
        fv1[o] = v1;
        fv2[o] = v2;
        fb[o] = bi;
      }
      if (fabs(cd) < pert) cd = (cd < 0.0) ? -pert : pert;
      // back substitution in place, then normalise
      double y2 = 0.0, y1 = bc / cd, nrm = y1 * y1;
      fb[(int64_t)(ka - 1) * k + t] = y1;
      for (int i = ka - 2; i >= 0; --i) {
        const int64_t o = (int64_t)i * k + t;
        const double y = (fb[o] - fv1[o] * y1 - fv2[o] * y2) / fu[o];
        fb[o] = y;
        nrm += y * y;
        y2 = y1;
        y1 = y;
      }
      const double s = 1.0 / sqrt(nrm);
      for (int i = 0; i < ka; ++i) fb[(int64_t)i * k + t] *= s;
    }
    __syncthreads();
    for (int t = tid; t < ka; t += NT) {
      if (t > 0 && lam[t] - lam[t - 1] <= ortol) continue;      // not a cluster leader
      int end = t + 1;
      while (end < ka && lam[end] - lam[end - 1] <= ortol) ++end;
      for (int sv = t + 1; sv < end; ++sv) {
        for (int r = t; r < sv; ++r) {
          double dot = 0.0;
          for (int i = 0; i < ka; ++i) dot += fb[(int64_t)i * k + r] * fb[(int64_t)i * k + sv];
          for (int i = 0; i < ka; ++i) fb[(int64_t)i * k + sv] -= dot * fb[(int64_t)i * k + r];
        }
        double nrm = 0.0;
        for (int i = 0; i < ka; ++i) nrm += fb[(int64_t)i * k + sv] * fb[(int64_t)i * k + sv];
        const double s = 1.0 / sqrt(nrm);
        for (int i = 0; i < ka; ++i) fb[(int64_t)i * k + sv] *= s;
      }
    }
    __syncthreads();
  }
}

// grid (ceil(k / 4), 1, B), 256 threads: wavefront w of block x owns eigenvector t = 4x + w
// and applies the reflectors H_{ka-3}, ..., H_0 to it (16 reflectors staged in LDS at a time).
__global__ void __launch_bounds__(256) tridiag_back_kernel(
    int32_t k, const int32_t *__restrict__ lock, const double *__restrict__ work, int64_t wstride,
    double *__restrict__ Zout, int32_t ldm) {
  constexpr int CH = 16;
  __shared__ double vs[CH][kMaxK];
  __shared__ double ts[CH];
  const int b = blockIdx.z;
  const int l = lock ? lock[b] : 0;
  const int ka = k - l;
  const int t0 = blockIdx.x * 4;
  if (ka <= 0 || t0 >= ka) return;
  const int tid = threadIdx.x, lane = tid & 63, t = t0 + (tid >> 6);
  const double *Wk = work + (int64_t)b * wstride;
  const double *refl = Wk, *tau = Wk + (int64_t)k * k;
  const double *fb = tau + k + 3 * (int64_t)k * k;
  double z[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    z[q] = (t < ka && i < ka) ? fb[(int64_t)i * k + t] : 0.0;
  }
  for (int j1 = ka - 3; j1 >= 0; j1 -= CH) {
    const int j0 = max(0, j1 - CH + 1), nj = j1 - j0 + 1;
    __syncthreads();
    for (int e = tid; e < nj * ka; e += 256) {
      const int jj = e / ka, c = e - jj * ka, j = j0 + jj;
      vs[jj][c] = (c > j) ? refl[(int64_t)j * k + c] : 0.0;
    }
    if (tid < nj) ts[tid] = tau[j0 + tid];
    __syncthreads();
    if (t < ka) {
      for (int jj = nj - 1; jj >= 0; --jj) {
        double dot = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = lane + 64 * q;
          if (i < ka) dot += vs[jj][i] * z[q];
        }
        const double s = ts[jj] * wave_sum(dot);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = lane + 64 * q;
          if (i < ka) z[q] -= s * vs[jj][i];
        }
      }
    }
  }
  if (t < ka) {
    double *Zb = Zout + (int64_t)b * ldm * ldm + (int64_t)t * ldm;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (i < ka) Zb[i] = z[q];
    }
  }
}

hipError_t tridiag_eig(int B, int32_t k, const int32_t *lock, const double *G, double *Z,
                       int32_t ldm, double *theta, int32_t *flag, double *scratch, double *work,
                       hipStream_t st) {
  if (B <= 0 || k <= 0) return hipSuccess;
  const int64_t ws = tridiag_work_elems(k);
  // per problem: the packed matrix in LDS when its active width fits, else global scratch
  tridiag_eig_kernel<true><<<B, 512, 0, st>>>(k, lock, G, ldm, theta, flag, scratch, work, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  tridiag_back_kernel<<<dim3((unsigned)ceil_div(k, 4), 1, (unsigned)B), 256, 0, st>>>(
      k, lock, work, ws, Z, ldm);
  return hipGetLastError();
}

}  // namespace scsf
