// Device-side evaluation of the operators' rows (5-point faces, 9-point Q1 cells, CSR).
#pragma once
#include "common.h"

namespace scsf {

// Bilinear element on the unit square, local node a = ax + 2 ay with (ax, ay) in {0,1}^2.
// d(phi_a)/dx = sx_a * (ay ? y : 1-y), d(phi_a)/dy = sy_a * (ax ? x : 1-x), sx = 2ax-1, sy = 2ay-1;
// the 1-D integrals are int (1-t)^2 = int t^2 = 1/3, int t(1-t) = 1/6, int t = int (1-t) = 1/2.
__device__ inline double q1_stiffness(const double *kc, int a, int b) {
  const int ax = a & 1, ay = a >> 1, bx = b & 1, by = b >> 1;
  const double sxa = 2 * ax - 1, sya = 2 * ay - 1, sxb = 2 * bx - 1, syb = 2 * by - 1;
  const double ixx = sxa * sxb * (ay == by ? 1.0 / 3.0 : 1.0 / 6.0);
  const double iyy = sya * syb * (ax == bx ? 1.0 / 3.0 : 1.0 / 6.0);
  const double ixy = 0.25 * (sxa * syb + sxb * sya);
  return kc[0] * ixx + kc[2] * iyy + kc[1] * ixy;
}

// 9-point coefficients of node (iy, ix): c9[(dy+1)*3 + (dx+1)] couples it to (iy+dy, ix+dx).
// The node is corner 3 of cell (iy, ix), 2 of (iy, ix+1), 1 of (iy+1, ix), 0 of (iy+1, ix+1);
// corner b of cell (cy, cx) is node (cy-1 + (b>>1), cx-1 + (b&1)).
__device__ inline void stencil9_coeffs(const OpDev &op, int iy, int ix, double c9[9]) {
  const int N = op.N;
  const double h = 1.0 / (N + 1);
  const double inv_h2 = 1.0 / (h * h);
#pragma unroll
  for (int t = 0; t < 9; ++t) c9[t] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cy = iy + (q >> 1), cx = ix + (q & 1);
    const int a = 3 - q;
    const double *kc = op.cell + ((int64_t)cy * (N + 1) + cx) * 3;
#pragma unroll
    for (int bl = 0; bl < 4; ++bl) {
      const int dy = (cy - 1 + (bl >> 1)) - iy;
      const int dx = (cx - 1 + (bl & 1)) - ix;
      c9[(dy + 1) * 3 + (dx + 1)] += q1_stiffness(kc, a, bl) * inv_h2;
    }
  }
}

// (A x)_p and the Gershgorin radius sum_q |A_pq| (q != p) plus A_pp.
template <int KIND>
__device__ inline double op_row(const OpDev &op, int64_t p, const double *x, double *gersh,
                                double *gersh_lo = nullptr) {
  if constexpr (KIND == SCSF_STENCIL5) {
    const int N = op.N;
    const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
    const double cw = op.wx[(int64_t)iy * (N + 1) + ix];
    const double ce = op.wx[(int64_t)iy * (N + 1) + ix + 1];
    const double cs = op.wy[(int64_t)iy * N + ix];
    const double cn = op.wy[(int64_t)(iy + 1) * N + ix];
    const double cd = cw + ce + cs + cn + (op.v ? op.v[p] : 0.0);
    double r = cd * x[p], g = cd;
    if (ix > 0) { r -= cw * x[p - 1]; g += fabs(cw); }
    if (ix < N - 1) { r -= ce * x[p + 1]; g += fabs(ce); }
    if (iy > 0) { r -= cs * x[p - N]; g += fabs(cs); }
    if (iy < N - 1) { r -= cn * x[p + N]; g += fabs(cn); }
    if (gersh) *gersh = g;
    if (gersh_lo) *gersh_lo = 2.0 * cd - g;
    return r;
  } else if constexpr (KIND == SCSF_STENCIL9) {
    const int N = op.N;
    const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
    double c9[9];
    stencil9_coeffs(op, iy, ix, c9);
    double r = 0.0, g = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      if (iy + dy >= 0 && iy + dy < N && ix + dx >= 0 && ix + dx < N) {
        r += c9[t] * x[p + dy * N + dx];
        g += (t == 4) ? c9[t] : fabs(c9[t]);
      }
    }
    if (gersh) *gersh = g;
    if (gersh_lo) *gersh_lo = 2.0 * c9[4] - g;
    return r;
  } else if constexpr (KIND == SCSF_PLATE) {
    // row p of S L diag(D) L S (S = diag(rho^-1/2), L = 5-point Dirichlet Laplacian / h^2):
    // the 13 coefficients gathered on the 5 x 5 offset square around p
    const int N = op.N;
    const int iy = (int)(p / N), ix = (int)(p - (int64_t)iy * N);
    const double ih2 = (double)(N + 1) * (double)(N + 1);
    const int oy[5] = {0, 0, 0, -1, 1}, ox[5] = {0, -1, 1, 0, 0};
    double c[25];
#pragma unroll
    for (int t = 0; t < 25; ++t) c[t] = 0.0;
    for (int u = 0; u < 5; ++u) {
      const int ky = iy + oy[u], kx = ix + ox[u];
      if (ky < 0 || ky >= N || kx < 0 || kx >= N) continue;
      const double dk = (u == 0 ? 4.0 : -1.0) * op.wx[(int64_t)ky * N + kx] * ih2 * ih2;
      for (int w = 0; w < 5; ++w) {
        const int jy = ky + oy[w], jx = kx + ox[w];
        if (jy < 0 || jy >= N || jx < 0 || jx >= N) continue;
        c[(oy[u] + oy[w] + 2) * 5 + (ox[u] + ox[w] + 2)] +=
            dk * (w == 0 ? 4.0 : -1.0) / sqrt(op.wy[(int64_t)jy * N + jx]);
      }
    }
    const double sp = 1.0 / sqrt(op.wy[p]);
    double r = 0.0, g = 0.0;
    for (int t = 0; t < 25; ++t) {
      if (c[t] == 0.0) continue;
      const int dy = t / 5 - 2, dx = t % 5 - 2;
      r += c[t] * x[p + (int64_t)dy * N + dx];
      g += (t == 12) ? c[t] : fabs(c[t]);
    }
    if (gersh) *gersh = sp * g;
    if (gersh_lo) *gersh_lo = sp * (2.0 * c[12] - g);
    return sp * r;
  } else {
    double r = 0.0, g = 0.0, d = 0.0;
    for (int32_t q = op.row_ptr[p]; q < op.row_ptr[p + 1]; ++q) {
      const int32_t c = op.col_idx[q];
      r += op.val[q] * x[c];
      g += (c == p) ? op.val[q] : fabs(op.val[q]);
      if (c == p) d += op.val[q];
    }
    if (gersh) *gersh = g;
    if (gersh_lo) *gersh_lo = 2.0 * d - g;
    return r;
  }
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the multiply-xor bijection.
__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Two standard normals (Box-Muller) for counter (idx, stream, tag) and a 64-bit seed.
__device__ inline double2 gauss2(uint64_t seed, uint64_t idx, uint32_t stream, uint32_t tag) {
  const uint4 r = philox4x32_10(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), stream, tag),
                                make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
  const uint64_t a = ((uint64_t)r.y << 32) | r.x, bb = ((uint64_t)r.w << 32) | r.z;
  const double u1 = ((a >> 11) + 1) * 0x1.0p-53;      // (0, 1]
  const double u2 = (bb >> 11) * 0x1.0p-53;           // [0, 1)
  const double rad = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  return make_double2(rad * c, rad * s);
}

}  // namespace scsf
