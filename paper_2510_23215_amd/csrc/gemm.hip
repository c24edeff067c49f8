// Tall-skinny FP64 products on the MFMA units of gfx950 (v_mfma_f64_16x16x4_f64).
//
//   gemm_tn : C = A^T B, A and B n x k blocks (n >> k): the Gram matrices of CholeskyQR2, the
//             projection V^T X of block Gram-Schmidt and the Rayleigh quotient X^T (A X).
//   gemm_nn : Out = beta Out + alpha In M with a small k x k matrix M: X R^-1, the Ritz
//             rotation X W, and the Gram-Schmidt update X - V C.
//
// MFMA operand layout (one wavefront, 64 lanes, lane = i + 16*kk):
//   A operand (16 x 4): lane holds A[i = lane%16][kk = lane/16]
//   B operand (4 x 16): lane holds B[kk = lane/16][j = lane%16]
//   D (16 x 16, 4 doubles per lane): lane holds D[lane/16 + 4*v][lane%16], v = 0..3
//   (rows interleaved with stride 4; checked on gfx950 with an in-bounds probe)
// gemm_tn contracts over rows, so the contraction index may be permuted freely: lane
// (c, r) loads 4 consecutive rows 4r..4r+3 of column c as one 32-byte vector and feeds them
// to 4 successive MFMAs, which keeps every load a full 128-byte segment per column.
#include "common.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace scsf {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

enum TnSym : int32_t { TN_GENERAL = 0, TN_GRAM = 1, TN_SYMMETRISE = 2 };

// grid: x = T*T output tiles of 32 x 32 (T = ldc/32), y = row chunk, z = problem.
__global__ void __launch_bounds__(256) gemm_tn_kernel(
    int64_t n, int64_t ld, const double *__restrict__ A, int64_t bsA, int32_t modeA,
    const double *__restrict__ Bm, int64_t bsB, int32_t modeB, int32_t k,
    const int32_t *__restrict__ lock, int32_t sym, double *__restrict__ partial,
    int64_t pstride, int32_t ldc, const int32_t *__restrict__ gate, int32_t gate_mask,
    const int32_t *__restrict__ rows) {
  __shared__ double red[3][64][16];
  const int b = blockIdx.z, s = blockIdx.y;
  if (gate && !(gate[b] & gate_mask)) return;
  const int64_t nb = rows ? (int64_t)rows[b] : n;    // this problem's row count
  if ((int64_t)s * kGramChunk >= nb) return;         // chunk beyond it: never reduced
  const int T = ldc / 32;
  const int ti = blockIdx.x % T, tj = blockIdx.x / T;
  if (sym == TN_GRAM && ti > tj) return;
  int32_t a0, ka, b0, kb;
  col_range(modeA, k, lock, b, a0, ka);
  col_range(modeB, k, lock, b, b0, kb);
  if (ti * 32 >= ka || tj * 32 >= kb) return;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r4 = lane >> 4, c16 = lane & 15;
  const int64_t row_begin = (int64_t)s * kGramChunk;
  const int64_t row_end = min(nb, row_begin + kGramChunk);
  const double *Ab = A + (int64_t)b * bsA;
  const double *Bb = Bm + (int64_t)b * bsB;

  const double *pa[2];
  const double *pb[2];
  bool va[2], vb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ca = ti * 32 + h * 16 + c16, cb = tj * 32 + h * 16 + c16;
    va[h] = ca < ka;
    vb[h] = cb < kb;
    pa[h] = Ab + (int64_t)(a0 + (va[h] ? ca : 0)) * ld;
    pb[h] = Bb + (int64_t)(b0 + (vb[h] ? cb : 0)) * ld;
  }
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (v4d){0.0, 0.0, 0.0, 0.0};

  // each wave takes every 4th group of 16 rows of the chunk
  for (int64_t r0 = row_begin + wave * 16; r0 < row_end; r0 += 64) {
    const int64_t rr = r0 + 4 * r4;
    v4d fa[2], fb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v4d xa = (v4d){0.0, 0.0, 0.0, 0.0}, xb = (v4d){0.0, 0.0, 0.0, 0.0};
      if (rr < row_end) {
        if (va[h]) xa = *reinterpret_cast<const v4d *>(pa[h] + rr);
        if (vb[h]) xb = *reinterpret_cast<const v4d *>(pb[h] + rr);
      }
      // rows beyond n inside the last 4-row group contribute nothing
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (rr + t >= row_end) { xa[t] = 0.0; xb[t] = 0.0; }
      }
      fa[h] = xa;
      fb[h] = xb;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(fa[x][t], fb[y][t], acc[x][y]);
  }

  // sum the four waves' tiles and store the chunk's partial 32 x 32 tile
  if (wave > 0) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave - 1][lane][(x * 2 + y) * 4 + v] = acc[x][y][v];
  }
  __syncthreads();
  if (wave == 0) {
    double *P = partial + ((int64_t)b * gridDim.y + s) * pstride;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = (x * 2 + y) * 4 + v;
          const double val = acc[x][y][v] + red[0][lane][e] + red[1][lane][e] + red[2][lane][e];
          const int i = ti * 32 + x * 16 + r4 + 4 * v;
          const int j = tj * 32 + y * 16 + c16;
          P[i + (int64_t)j * ldc] = val;
        }
  }
}

// C_b(i, j) = sum over chunks (fixed order) of the partial tiles.
__global__ void gemm_tn_reduce_kernel(int32_t nchunks, int32_t chunk, int32_t modeA, int32_t modeB,
                                      int32_t k, const int32_t *__restrict__ lock, int32_t sym,
                                      const double *__restrict__ partial, int64_t pstride,
                                      double *__restrict__ C, int32_t ldc,
                                      const int32_t *__restrict__ gate, int32_t gate_mask,
                                      const int32_t *__restrict__ rows) {
  const int b = blockIdx.z;
  if (gate && !(gate[b] & gate_mask)) return;
  const int32_t nch = rows ? (int32_t)ceil_div((int64_t)rows[b], chunk) : nchunks;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ldc * ldc) return;
  int32_t a0, ka, b0, kb;
  col_range(modeA, k, lock, b, a0, ka);
  col_range(modeB, k, lock, b, b0, kb);
  const int i = (int)(e % ldc), j = (int)(e / ldc);
  if (i >= ka || j >= kb) return;
  const double *P = partial + (int64_t)b * nchunks * pstride;
  double v = 0.0;
  if (sym == TN_GRAM) {
    const int lo = min(i, j), hi = max(i, j);
    for (int s = 0; s < nch; ++s) v += P[(int64_t)s * pstride + lo + (int64_t)hi * ldc];
  } else if (sym == TN_SYMMETRISE) {
    double w = 0.0;
    for (int s = 0; s < nch; ++s) {
      v += P[(int64_t)s * pstride + i + (int64_t)j * ldc];
      w += P[(int64_t)s * pstride + j + (int64_t)i * ldc];
    }
    v = 0.5 * (v + w);
  } else {
    for (int s = 0; s < nch; ++s) v += P[(int64_t)s * pstride + i + (int64_t)j * ldc];
  }
  C[(int64_t)b * ldc * ldc + i + (int64_t)j * ldc] = v;
}

// ---- slab form for blocks up to 128 columns
// One workgroup of NW waves takes a row chunk of R rows of one problem and computes every 16 x
// 16 output tile of that chunk (the upper ones of a Gram matrix, all of a general product).
// Slabs of SR rows of all the problem's active columns are staged in LDS with coalesced 32-byte
// loads (each element read from HBM once per product), double-buffered so the loads of the next
// slab are in flight while the MFMAs run on this one.  Every wave has a compile-time list of
// tiles (round-robin over the tile list), keeps the 16 x 4 fragments of the columns its tiles
// need in registers for each 16-row group, and issues its MFMAs with the contraction index
// outermost, so consecutive MFMAs write different accumulators.  Tiles beyond a problem's
// active columns (locking) are skipped.  Partial tiles land in the same layout as the
// 32 x 32-tile kernel's, and the same reduction sums them.
template <class F, int... U>
__device__ inline void static_for_impl(F &&f, std::integer_sequence<int, U...>) {
  (f(std::integral_constant<int, U>{}), ...);
}
template <int N, class F> __device__ inline void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int KT, bool SYM> struct SlabTiles {   // KT x KT tiles; SYM: those with i <= j
  static constexpr int count() {
    int c = 0;
    for (int i = 0; i < KT; ++i)
      for (int j = 0; j < KT; ++j) c += (!SYM || i <= j) ? 1 : 0;
    return c;
  }
  static constexpr int at(int t) {               // i * 64 + j of tile t
    int c = 0;
    for (int i = 0; i < KT; ++i)
      for (int j = 0; j < KT; ++j)
        if (!SYM || i <= j) {
          if (c == t) return i * 64 + j;
          ++c;
        }
    return -1;
  }
  static constexpr uint32_t rows_of(int w, int nw) {   // bit i: tiles of wave w use A block i
    uint32_t m = 0;
    for (int t = w; t < count(); t += nw) m |= 1u << (at(t) / 64);
    return m;
  }
  static constexpr uint32_t cols_of(int w, int nw) {   // bit j: tiles of wave w use B block j
    uint32_t m = 0;
    for (int t = w; t < count(); t += nw) m |= 1u << (at(t) % 64);
    return m;
  }
};

template <int KT, bool SYM, int NW, int SR, int W>
__device__ inline void tn_slab_body(int64_t r_begin, int64_t r_end, int64_t ld, const double *Ab,
                                    const double *Bb, int ka, int kb, double *ldsA, double *ldsB,
                                    double *P, int ldc) {
  using TL = SlabTiles<KT, SYM>;
  constexpr int NT = TL::count();
  constexpr int TPW = (NT - W + NW - 1) / NW;            // tiles of this wave
  constexpr int CS = SR + 4;                             // padded LDS column stride
  constexpr int NQ = KT * 16 * (SR / 4);                 // 4-row quads per slab and operand
  constexpr int QPT = (NQ + NW * 64 - 1) / (NW * 64);
  constexpr uint32_t AM = SYM ? (TL::rows_of(W, NW) | TL::cols_of(W, NW)) : TL::rows_of(W, NW);
  constexpr uint32_t BM = SYM ? 0u : TL::cols_of(W, NW);
  const int tid = threadIdx.x, lane = tid & 63;
  const int r4 = lane >> 4, c16 = lane & 15;
  v4d acc[TPW > 0 ? TPW : 1];
  static_for<TPW>([&](auto u) { acc[u] = (v4d){0.0, 0.0, 0.0, 0.0}; });
  v4d sa[QPT], sb[SYM ? 1 : QPT];
  auto load1 = [&](const double *X, int kx, int u, int64_t s0) -> v4d {
    const int q = tid + NW * 64 * u;
    const int col = q / (SR / 4), rq = q % (SR / 4);
    const int64_t r = s0 + 4 * rq;
    v4d v = (v4d){0.0, 0.0, 0.0, 0.0};
    if (q < NQ && col < kx && r < r_end) {
      const double *src = X + (int64_t)col * ld + r;
      if (r + 3 < r_end) {
        v = *reinterpret_cast<const v4d *>(src);
      } else {
        for (int t = 0; t < 4; ++t) v[t] = (r + t < r_end) ? src[t] : 0.0;
      }
    }
    return v;
  };
  auto load = [&](int64_t s0) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) sa[u] = load1(Ab, ka, u, s0);
    if constexpr (!SYM) {
#pragma unroll
      for (int u = 0; u < QPT; ++u) sb[u] = load1(Bb, kb, u, s0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      const int q = tid + NW * 64 * u;
      if (q < NQ) {
        const int col = q / (SR / 4), rq = q % (SR / 4);
        const int o = buf * KT * 16 * CS + col * CS + 4 * rq;
        *reinterpret_cast<v4d *>(&ldsA[o]) = sa[u];
        if constexpr (!SYM) *reinterpret_cast<v4d *>(&ldsB[o]) = sb[u];
      }
    }
  };
  load(r_begin);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t s0 = r_begin; s0 < r_end; s0 += SR) {
    const bool more = s0 + SR < r_end;
    if (more) load(s0 + SR);
    const double *LA = ldsA + buf * KT * 16 * CS;
    const double *LB = SYM ? LA : ldsB + buf * KT * 16 * CS;
    for (int g = 0; g < SR / 16; ++g) {
      v4d fa[KT], fb[SYM ? 1 : KT];
      static_for<KT>([&](auto i) {
        if constexpr ((AM >> decltype(i)::value) & 1u)
          fa[i] = *reinterpret_cast<const v4d *>(&LA[(i * 16 + c16) * CS + g * 16 + 4 * r4]);
      });
      if constexpr (!SYM)
        static_for<KT>([&](auto j) {
          if constexpr ((BM >> decltype(j)::value) & 1u)
            fb[j] = *reinterpret_cast<const v4d *>(&LB[(j * 16 + c16) * CS + g * 16 + 4 * r4]);
        });
      static_for<4>([&](auto t) {
        constexpr int tt = decltype(t)::value;
        static_for<TPW>([&](auto u) {
          constexpr int ij = TL::at(W + NW * decltype(u)::value);
          constexpr int i = ij / 64, j = ij % 64;
          if constexpr (SYM) {
            acc[u] = mfma16x16x4(fa[i][tt], fa[j][tt], acc[u]);
          } else if (i * 16 < ka && j * 16 < kb) {   // widths differ: skip dead tiles
            acc[u] = mfma16x16x4(fa[i][tt], fb[j][tt], acc[u]);
          }
        });
      });
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  static_for<TPW>([&](auto u) {
    constexpr int ij = TL::at(W + NW * decltype(u)::value);
    constexpr int i = ij / 64, j = ij % 64;
    {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[(i * 16 + r4 + 4 * v) + (int64_t)(j * 16 + c16) * ldc] = acc[u][v];
    }
  });
}

// grid: x = row chunk of R rows, z = problem.
// Gram form: two workgroups of 8 waves share a CU (73.7 KB of LDS each), so each wave gets at
// most 128 registers (4 waves per SIMD); the general form runs one workgroup per CU.
template <int KT, bool SYM, int NW, int SR>
__global__ void __launch_bounds__(NW * 64, SYM ? 4 : 2) gemm_tn_slab_kernel(
    int64_t n, int64_t ld, const double *__restrict__ A, int64_t bsA, int32_t modeA,
    const double *__restrict__ Bm, int64_t bsB, int32_t modeB, int32_t k,
    const int32_t *__restrict__ lock, int32_t R, double *__restrict__ partial, int64_t pstride,
    int32_t ldc, const int32_t *__restrict__ gate, int32_t gate_mask,
    const int32_t *__restrict__ rows) {
  constexpr int CS = SR + 4;
  __shared__ double ldsA[2 * KT * 16 * CS];
  __shared__ double ldsB[SYM ? 1 : 2 * KT * 16 * CS];
  const int b = blockIdx.z, s = blockIdx.x;
  if (gate && !(gate[b] & gate_mask)) return;
  const int64_t nb = rows ? (int64_t)rows[b] : n;
  const int64_t r_begin = (int64_t)s * R;
  if (r_begin >= nb) return;                           // chunk beyond it: never reduced
  const int64_t r_end = min(nb, r_begin + R);
  int32_t a0, ka, b0, kb;
  col_range(modeA, k, lock, b, a0, ka);
  col_range(modeB, k, lock, b, b0, kb);
  if (ka <= 0 || kb <= 0) return;
  const double *Ab = A + (int64_t)b * bsA + (int64_t)a0 * ld;
  const double *Bb = Bm + (int64_t)b * bsB + (int64_t)b0 * ld;
  double *P = partial + ((int64_t)b * gridDim.x + s) * pstride;
  const int w = threadIdx.x >> 6;
  // the body for this problem's active width (16-column blocks), so locked columns cost no
  // MFMAs and no tile carries a per-tile test
  const int kt = (int)ceil_div((int64_t)max(ka, kb), 16);
  static_for<KT>([&](auto KM1) {
    constexpr int KW = decltype(KM1)::value + 1;
    if (kt == KW)
      static_for<NW>([&](auto W) {
        if (w == decltype(W)::value)
          tn_slab_body<KW, SYM, NW, SR, decltype(W)::value>(r_begin, r_end, ld, Ab, Bb, ka, kb,
                                                            ldsA, ldsB, P, ldc);
      });
  });
}

constexpr int kSlabChunkGram = 512;      // rows per workgroup, Gram form
constexpr int kSlabChunkGeneral = 512;   // rows per workgroup, general form
constexpr int kSlabNW = 8;               // waves per workgroup

template <int KT>
static void launch_slab_kt(bool gram, int B, int64_t n, int64_t ld, const double *A, int64_t bsA,
                           int32_t modeA, const double *Bm, int64_t bsB, int32_t modeB, int32_t k,
                           const int32_t *lock, double *partial, int64_t pstride, int32_t ldc,
                           const int32_t *gate, int32_t gate_mask, const int32_t *rows,
                           hipStream_t st) {
  if (gram) {
    dim3 g((unsigned)ceil_div(n, kSlabChunkGram), 1, (unsigned)B);
    gemm_tn_slab_kernel<KT, true, kSlabNW, 32><<<g, kSlabNW * 64, 0, st>>>(
        n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, kSlabChunkGram, partial, pstride, ldc,
        gate, gate_mask, rows);
  } else {
    dim3 g((unsigned)ceil_div(n, kSlabChunkGeneral), 1, (unsigned)B);
    gemm_tn_slab_kernel<KT, false, kSlabNW, 16><<<g, kSlabNW * 64, 0, st>>>(
        n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, kSlabChunkGeneral, partial, pstride, ldc,
        gate, gate_mask, rows);
  }
}

// The slabs' LDS is sized for the launch's width (KT = 4, 5, 6 or 8 blocks of 16 columns), so
// narrow blocks leave room on the CU for other lanes' work.
static void launch_slab(bool gram, int B, int64_t n, int64_t ld, const double *A, int64_t bsA,
                        int32_t modeA, const double *Bm, int64_t bsB, int32_t modeB, int32_t k,
                        const int32_t *lock, double *partial, int64_t pstride, int32_t ldc,
                        const int32_t *gate, int32_t gate_mask, const int32_t *rows,
                        hipStream_t st) {
  const int kt = (int)ceil_div(k, 16);
  if (kt <= 4)
    launch_slab_kt<4>(gram, B, n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, partial, pstride,
                      ldc, gate, gate_mask, rows, st);
  else if (kt == 5)
    launch_slab_kt<5>(gram, B, n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, partial, pstride,
                      ldc, gate, gate_mask, rows, st);
  else if (kt == 6)
    launch_slab_kt<6>(gram, B, n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, partial, pstride,
                      ldc, gate, gate_mask, rows, st);
  else
    launch_slab_kt<8>(gram, B, n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, partial, pstride,
                      ldc, gate, gate_mask, rows, st);
}

int64_t gemm_tn_partial_elems(int64_t n, int32_t ldc) {
  // room for the most chunks any form uses (the general slab form's 512-row chunks)
  return ceil_div(n, std::min(kGramChunk, kSlabChunkGeneral)) * (int64_t)ldc * ldc;
}

hipError_t gemm_tn(int B, int64_t n, int64_t ld, const double *A, int64_t bsA, int32_t modeA,
                   const double *Bm, int64_t bsB, int32_t modeB, int32_t k, const int32_t *lock,
                   bool symmetric, double *partial, int64_t partial_stride, double *C, int32_t ldc,
                   const int32_t *gate, int32_t gate_mask, hipStream_t st, const int32_t *rows) {
  if (B <= 0 || n <= 0) return hipSuccess;
  const int32_t sym = symmetric ? (A == Bm && modeA == modeB ? TN_GRAM : TN_SYMMETRISE)
                                : TN_GENERAL;
  const int KT = (int)ceil_div(k, 16);
  int32_t chunk, nchunks;
  if (KT <= 8) {                         // slab form: up to 128 columns
    const bool gram = sym == TN_GRAM;
    chunk = gram ? kSlabChunkGram : kSlabChunkGeneral;
    nchunks = (int32_t)ceil_div(n, chunk);
    launch_slab(gram, B, n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, partial,
                partial_stride / nchunks, ldc, gate, gate_mask, rows, st);
  } else {                               // 32 x 32 tiles per workgroup
    chunk = kGramChunk;
    nchunks = (int32_t)ceil_div(n, chunk);
    const int T = ldc / 32;
    dim3 g1((unsigned)(T * T), (unsigned)nchunks, (unsigned)B);
    gemm_tn_kernel<<<g1, 256, 0, st>>>(n, ld, A, bsA, modeA, Bm, bsB, modeB, k, lock, sym,
                                       partial, partial_stride / nchunks, ldc, gate, gate_mask,
                                       rows);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  dim3 g2((unsigned)ceil_div((int64_t)ldc * ldc, 256), 1, (unsigned)B);
  gemm_tn_reduce_kernel<<<g2, 256, 0, st>>>(nchunks, chunk, modeA, modeB, k, lock, sym, partial,
                                            partial_stride / nchunks, C, ldc, gate, gate_mask,
                                            rows);
  return hipGetLastError();
}

// grid: x = row tiles of 64 (4 waves x 16 rows), z = problem.  A body computes NT tiles of 16
// output columns (compile-time, so the MFMA loop carries no per-tile test and M is staged only
// as wide as the body); columns past the problem's output width come out zero and are not
// stored.
// MODE 0: Out = In M;  MODE 1: Out -= In M;  MODE 2: Out = beta Out + alpha In M.  The first two
// (every call of the solvers) are compile-time: a runtime alpha in the epilogue alone took 56
// more registers.
template <int NT, int MODE>
__device__ inline void gemm_nn_body(int64_t nb, int64_t ld, const double *Ib, double *Ob, int ki,
                                    int ko, const double *Mb, int32_t ldm, double alpha,
                                    double beta, double *Ms) {
  constexpr int KC = 32;                       // rows of M staged per pass
  constexpr int MS = NT * 16 + 2;              // padded LDS row stride
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r4 = lane >> 4, c16 = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t row = row0 + c16;
  const bool row_ok = row < nb;
  v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (int kk0 = 0; kk0 < ki; kk0 += KC) {
    __syncthreads();
    for (int e = threadIdx.x; e < KC * NT * 16; e += 256) {
      const int r = e % KC, c = e / KC;          // consecutive threads read down a column of M
      const int kk = kk0 + r;
      Ms[r * MS + c] = (kk < ki && c < ko) ? Mb[kk + (int64_t)c * ldm] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < KC; t += 4) {
      const int kk = kk0 + t + r4;
      const double bf = (row_ok && kk < ki) ? Ib[(int64_t)kk * ld + row] : 0.0;
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        const double af = Ms[(t + r4) * MS + ct * 16 + c16];
        acc[ct] = mfma16x16x4(af, bf, acc[ct]);
      }
    }
  }
  if (!row_ok) return;
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = ct * 16 + r4 + 4 * v;
      if (col < ko) {
        double *o = Ob + (int64_t)col * ld + row;
        if constexpr (MODE == 0) *o = acc[ct][v];
        else if constexpr (MODE == 1) *o -= acc[ct][v];
        else *o = (beta == 0.0) ? alpha * acc[ct][v] : beta * (*o) + alpha * acc[ct][v];
      }
    }
  }
}

// NTMAX = ceil(k / 16) is chosen on the host; a workgroup whose problem has at most half of
// that width active (locked columns) runs the half-width body.  Two bodies keep the kernel as
// lean in registers as a single one (a body per width raised it from 108 to 164 VGPRs at 8
// tiles and cost a quarter of the speed).
template <int NTMAX, int MODE>
__global__ void __launch_bounds__(256) gemm_nn_kernel(
    int64_t n, int64_t ld, const double *In, int64_t bsI, int32_t modeI, double *Out,
    int64_t bsO, int32_t modeO, int32_t k, const int32_t *__restrict__ lock,
    const double *__restrict__ M, int32_t ldm, double alpha, double beta,
    const int32_t *__restrict__ gate, int32_t gate_mask, const int32_t *__restrict__ skip,
    int32_t skip_mask, const int32_t *__restrict__ rows) {
  __shared__ double Ms[32 * (NTMAX * 16 + 2)];
  const int b = blockIdx.z;
  if (gate && !(gate[b] & gate_mask)) return;
  if (skip && (skip[b] & skip_mask)) return;
  int32_t i0, ki, o0, ko;
  col_range(modeI, k, lock, b, i0, ki);
  col_range(modeO, k, lock, b, o0, ko);
  if (ko <= 0) return;
  if (ki <= 0 && beta == 1.0) return;          // nothing to add
  const int64_t nb = rows ? (int64_t)rows[b] : n;
  if ((int64_t)blockIdx.x * 64 >= nb) return;  // row tile beyond this problem's rows
  const double *Ib = In + (int64_t)b * bsI + (int64_t)i0 * ld;
  double *Ob = Out + (int64_t)b * bsO + (int64_t)o0 * ld;
  const double *Mb = M + (int64_t)b * ldm * ldm;
  constexpr int HALF = (NTMAX + 1) / 2;
  if ((ko + 15) / 16 <= HALF)
    gemm_nn_body<HALF, MODE>(nb, ld, Ib, Ob, ki, ko, Mb, ldm, alpha, beta, Ms);
  else
    gemm_nn_body<NTMAX, MODE>(nb, ld, Ib, Ob, ki, ko, Mb, ldm, alpha, beta, Ms);
}

hipError_t gemm_nn(int B, int64_t n, int64_t ld, const double *In, int64_t bsI, int32_t modeI,
                   double *Out, int64_t bsO, int32_t modeO, int32_t k, const int32_t *lock,
                   const double *M, int32_t ldm, double alpha, double beta, const int32_t *gate,
                   int32_t gate_mask, const int32_t *skip, int32_t skip_mask, hipStream_t st,
                   const int32_t *rows) {
  if (B <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;
  dim3 grid((unsigned)ceil_div(n, 64), 1, (unsigned)B);
  const int nt = (int)ceil_div(k, 16);
  const int mode = (alpha == 1.0 && beta == 0.0) ? 0 : (alpha == -1.0 && beta == 1.0) ? 1 : 2;
  switch (nt) {
#define SCSF_NN_MODE(T, MD)                                                                     \
  gemm_nn_kernel<T, MD><<<grid, 256, 0, st>>>(n, ld, In, bsI, modeI, Out, bsO, modeO, k, lock, M, \
                                              ldm, alpha, beta, gate, gate_mask, skip,          \
                                              skip_mask, rows)
#define SCSF_NN(T)                                                                              \
  case T:                                                                                      \
    if (mode == 0) SCSF_NN_MODE(T, 0);                                                         \
    else if (mode == 1) SCSF_NN_MODE(T, 1);                                                    \
    else SCSF_NN_MODE(T, 2);                                                                   \
    break;
    SCSF_NN(1) SCSF_NN(2) SCSF_NN(3) SCSF_NN(4) SCSF_NN(5) SCSF_NN(6) SCSF_NN(7) SCSF_NN(8)
    SCSF_NN(9) SCSF_NN(10) SCSF_NN(11) SCSF_NN(12) SCSF_NN(13) SCSF_NN(14) SCSF_NN(15) SCSF_NN(16)
#undef SCSF_NN
#undef SCSF_NN_MODE
    default: break;
  }
  return hipGetLastError();
}

}  // namespace scsf
