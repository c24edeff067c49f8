// Host side of libscsf: handle and workspace, the batched ChFSI engine (Algorithm 3), the step
// primitives, the sort (Algorithm 2) and the chunked, warm-started sequence solver.
//
// The engine runs B independent problems of the same shape in lockstep: every kernel of an
// outer iteration is one launch over all B problems (grid z = problem), and each problem's
// active column range [lock[b], k) is read on the device, so problems at different stages of
// convergence share the launches.  The host synchronises once per outer iteration to read the
// lock counts.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "cnn.h"
#include "common.h"

using namespace scsf;

namespace {

enum BufId {
  B_X, B_Y1, B_Y2, B_W, B_G, B_M, B_PART, B_THETA, B_RES, B_INT, B_BND, B_COEF, B_UNIT, B_CHOL,
  B_JAC, B_LZ, B_OPS, B_WIN, B_SORTF, B_SORTD, B_SORTO, B_REC, B_RANK, B_E32, B_R32, B_SRC,
  B_GAIN, B_WINB, B_HINT, B_MDEG, B_NETF, B_NETH, B_NETD, B_ROWS, B_EIG, B_CDEG, B_SQT, B_SQP, B_COEF2,
  B_TEV, B_TVV, B_NETL, B_PREOPS, B_PRELZ, B_PREBND, B_SORTV, B_COUNT
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool in_arena = false;                 // carved from a caller-owned workspace
  uint64_t gen = 0;                      // arena generation it was carved in
};

// A caller-owned device workspace (scsf_set_workspace).  While one is set, every device
// buffer is carved from it by a bump pointer: at the start of each top-level entry point the
// pointer returns to the base (nothing the library keeps lives across calls), and a buffer
// that must grow is carved anew.  A call that needs more than `cap` returns SCSF_ENOMEM.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  size_t peak = 0;
  uint64_t gen = 1;
  int depth = 0;                         // nesting of entry points (reset at depth 0 only)
  std::mutex mu;                         // the lanes carve concurrently
};

// Per-phase device times (Algorithm 3's steps), from HIP events on a lane's stream.
enum Phase { PH_FILTER, PH_ORTH, PH_RR, PH_RESID, PH_BOUND, PH_COUNT };

// Device buffers, pinned host staging, a stream and filter timing of one concurrent lane.
struct Workspace {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena *arena = nullptr;
  DevBuf bufs[B_COUNT];
  double phase_ms[PH_COUNT] = {0, 0, 0, 0, 0};   // accumulated (scsf_profile_read)
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  bool prof = false;                     // filter-launch timing (scsf_profile_*)
  std::vector<hipEvent_t> ev;            // 2 per pending launch
  std::vector<double> ev_bytes;          // algorithmic bytes of each pending timed span
  std::vector<int> ev_count;             // filter launches inside each pending timed span
  int ev_used = 0;
  scsf_profile acc{};
};

}  // namespace

struct scsf_handle {
  int device = 0;
  int lanes = 4;                         // concurrent chain groups in scsf_solve_sequence
  bool graphs = true;                    // outer iterations of chained solves as HIP graphs
  int eig = SCSF_EIG_JACOBI;             // Rayleigh-Ritz eigensolver
  int fuse = 0;                          // Chebyshev steps per fused filter launch (0: one)
  int batch_form = SCSF_BATCH_GROUPED;   // uneven batches: per-group batches or one sweep
  // autotuned settings: SpMM columns per thread per (k bucket, n bucket), block width per L
  int32_t cpt[4][3] = {{4, 4, 4}, {4, 4, 4}, {4, 4, 4}, {4, 4, 4}};
  std::vector<std::pair<int32_t, int32_t>> widths;
  std::vector<Workspace *> ws;           // ws[0] runs on the caller's stream; ws[1..] are the
                                         // lanes of chained solves (private streams)
  Arena arena;                           // caller-owned workspace (base == nullptr: none)
};

namespace {

#define HIPCHK(x)                               \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return SCSF_EHIP;     \
  } while (0)
#define STCHK(x)                                \
  do {                                          \
    int s_ = (x);                               \
    if (s_ != SCSF_OK) return s_;               \
  } while (0)

template <typename T>
int grow(Workspace *h, int id, size_t count, T **out) {
  DevBuf &b = h->bufs[id];
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  Arena *a = h->arena;
  if (a && a->base) {
    std::lock_guard<std::mutex> lk(a->mu);
    if (!(b.in_arena && b.gen == a->gen && b.bytes >= bytes)) {
      const size_t off = (a->used + 255) / 256 * 256;
      if (off > a->cap || bytes > a->cap - off) return SCSF_ENOMEM;
      b.p = a->base + off;
      b.bytes = bytes;
      b.in_arena = true;
      b.gen = a->gen;
      a->used = off + bytes;
      a->peak = std::max(a->peak, a->used);
    }
    *out = static_cast<T *>(b.p);
    return SCSF_OK;
  }
  if (b.in_arena) {                      // left over from a workspace that was removed
    b.p = nullptr;
    b.bytes = 0;
    b.in_arena = false;
  }
  if (b.bytes < bytes) {
    if (b.p) {
      if (hipStreamSynchronize(h->stream) != hipSuccess) return SCSF_EHIP;
      if (hipFree(b.p) != hipSuccess) return SCSF_EHIP;
      b.p = nullptr;
      b.bytes = 0;
    }
    const size_t nb = bytes + bytes / 8;
    if (hipMalloc(&b.p, nb) != hipSuccess) {
      b.p = nullptr;
      return SCSF_ENOMEM;
    }
    b.bytes = nb;
  }
  *out = static_cast<T *>(b.p);
  return SCSF_OK;
}

int grow_pinned(Workspace *h, size_t bytes) {
  if (h->pinned_bytes >= bytes) return SCSF_OK;
  if (h->pinned) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return SCSF_EHIP;
    (void)hipHostFree(h->pinned);
    h->pinned = nullptr;
    h->pinned_bytes = 0;
  }
  if (hipHostMalloc(&h->pinned, bytes, hipHostMallocDefault) != hipSuccess) return SCSF_ENOMEM;
  h->pinned_bytes = bytes;
  return SCSF_OK;
}

int check_op(const scsf_operator *A) {
  if (!A || A->n <= 0) return SCSF_EINVAL;
  if (A->kind == SCSF_STENCIL5) {
    if (A->nx <= 0 || (int64_t)A->nx * A->nx != A->n || !A->wx || !A->wy) return SCSF_EINVAL;
  } else if (A->kind == SCSF_STENCIL9) {
    if (A->nx <= 0 || (int64_t)A->nx * A->nx != A->n || !A->cell) return SCSF_EINVAL;
  } else if (A->kind == SCSF_CSR) {
    if (!A->row_ptr || !A->col_idx || !A->val || A->nnz < 0) return SCSF_EINVAL;
  } else if (A->kind == SCSF_PLATE) {
    if (A->nx <= 0 || A->nx > 600 || (int64_t)A->nx * A->nx != A->n || !A->wx || !A->wy || A->v)
      return SCSF_EINVAL;
  } else {
    return SCSF_EINVAL;
  }
  if (A->n > ((int64_t)1 << 31) - 64) return SCSF_EINVAL;
  return SCSF_OK;
}

// The plate family runs in FP64 only.
int check_op_precision(const scsf_operator &A, const scsf_params *p) {
  return (A.kind == SCSF_PLATE && p->precision != SCSF_FP64) ? SCSF_EINVAL : SCSF_OK;
}

OpDev to_dev(const scsf_operator &A) {
  OpDev d;
  d.kind = A.kind;
  d.N = A.nx;
  d.n = A.n;
  d.wx = A.wx;
  d.wy = A.wy;
  d.v = A.v;
  d.cell = A.cell;
  d.row_ptr = A.row_ptr;
  d.col_idx = A.col_idx;
  d.val = A.val;
  return d;
}

// Event pairs are recorded around each filter launch and drained at the next
// synchronisation point (no extra synchronisation is added).
int prof_begin(Workspace *h, double bytes, int launches = 1) {
  if (!h->prof) return -1;
  if ((size_t)(2 * h->ev_used + 2) > h->ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      h->ev.push_back(e);
    }
  }
  const int slot = h->ev_used++;
  if ((size_t)slot >= h->ev_bytes.size()) {
    h->ev_bytes.resize(slot + 1);
    h->ev_count.resize(slot + 1);
  }
  h->ev_bytes[slot] = bytes;
  h->ev_count[slot] = launches;
  if (hipEventRecord(h->ev[2 * slot], h->stream) != hipSuccess) return -1;
  return slot;
}
void prof_end(Workspace *h, int slot) {
  if (slot >= 0) (void)hipEventRecord(h->ev[2 * slot + 1], h->stream);
}
void prof_drain(Workspace *h) {  // call only after the stream was synchronised
  for (int i = 0; i < h->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess) {
      h->acc.filter_launches += h->ev_count[i];
      h->acc.filter_ms += ms;
      h->acc.filter_bytes += h->ev_bytes[i];
    }
  }
  h->ev_used = 0;
}

// ------------------------------------------------------------------------------- the engine
struct Engine {
  Workspace *h = nullptr;
  hipStream_t st = nullptr;
  int B = 0;
  int64_t n = 0, ld = 0, bs = 0;
  int32_t k = 0, L = 0, m = 0, kind = 0, ldm = 0, lz_steps = 20;
  double tol = 1e-8;
  uint64_t seed = 0;
  int64_t part_stride = 0;
  double *X = nullptr, *Y1 = nullptr, *Y2 = nullptr, *W = nullptr, *G = nullptr, *M = nullptr;
  double *part = nullptr, *theta = nullptr, *res = nullptr, *bnd = nullptr, *coef = nullptr;
  double *unit = nullptr, *chol = nullptr, *jac = nullptr, *lz = nullptr, *rec = nullptr;
  int32_t *ranks = nullptr, *nsweeps = nullptr;
  // mixed precision (FP32 filter in residual form)
  bool mixed = false, w_stale = true;
  // per-problem filter degrees (hinted sequences) and window hints
  bool var_deg = false;
  // adaptive filter: per-column degrees in [m_base, m] (m = min(2 m_base, 64)), computed on
  // the device after every iteration; mdeg[b] holds their maximum
  bool adaptive = false;
  int32_t m_base = 0;
  int32_t *cdeg = nullptr, *h_cdeg = nullptr;
  // smallest-magnitude mode: the filter polynomial is in A^2 (each step applies A twice, with
  // T = A Y_i and the non-operator terms P in two extra blocks); Rayleigh-Ritz, residuals and
  // locking stay with A, the pairs ordered by |theta|
  bool mag = false;
  double *T = nullptr, *P = nullptr, *coef2 = nullptr;
  // smallest magnitude from the lower end: the plain filter, locking until the lowest
  // converged pairs hold L with |theta| <= their largest (lock_kernel mode 2); extract()
  // returns those L ordered by |theta|; flag bit 16 marks a problem whose block ran out of
  // pairs first (not certified)
  bool mag_low = false;
  // fused filter: groups of `fuse` Chebyshev steps per launch (0 = one step per launch); only
  // for the plain FP64 filter of the grid stencils (fused_filter())
  int fuse = 0;
  // adaptive: per problem, the filter columns (sum of column degrees) and the largest column
  // degree of the last iteration
  std::vector<int64_t> it_cols;
  std::vector<int32_t> it_deg;
  int32_t *mdeg = nullptr, *h_mdeg = nullptr, *h_mraw = nullptr;
  double *hint = nullptr, *h_hint = nullptr;
  int32_t mcur = 0;                      // degree of the current iteration (max over problems)
  float *E32[3] = {nullptr, nullptr, nullptr}, *R32 = nullptr;
  double *src = nullptr, *gain = nullptr, *winb = nullptr;
  int32_t *lock = nullptr, *nconv = nullptr, *done = nullptr, *flag = nullptr, *need = nullptr;
  // per-slot widths (one lockstep batch over problems of different (L, k)): slot b's problem
  // owns columns [off_b, k) of the k-wide block (off_b = k - k_b) and wants L_b pairs; its
  // columns below off_b are zero, locked from the start, and only the locking, the window's
  // lowest Ritz value and the extraction look at off_b
  bool varw = false;
  int32_t *offv = nullptr, *Lv = nullptr, *h_off = nullptr, *h_Lv = nullptr;
  int32_t off(int b) const { return varw ? h_off[b] : 0; }
  int32_t Lof(int b) const { return varw ? h_Lv[b] : L; }
  OpDev *ops = nullptr;
  int32_t *rows = nullptr, *h_rows = nullptr;   // per-problem row count (uneven batches)
  int cpt = 2;                                  // filter-step tile (autotuned)
  int32_t Nmax = 0;                             // largest grid side the engine is sized for
  bool pot = true;                              // some operator it runs may have a potential
  int eig = SCSF_EIG_JACOBI;                    // Rayleigh-Ritz eigensolver
  double *eigw = nullptr;                       // its work area
  // pinned host mirrors
  int32_t *h_lock = nullptr, *h_nconv = nullptr, *h_done = nullptr, *h_flag = nullptr;
  int32_t *h_need = nullptr, *h_perm = nullptr;
  double *h_theta = nullptr, *h_res = nullptr, *h_bnd = nullptr, *h_unit = nullptr;
  double *h_vals = nullptr;              // extraction: each slot's sorted values (B*k)
  int32_t *perm_d = nullptr;             // extraction: each slot's column order (device, B*k)
  double *vals_d = nullptr;              // extraction: each slot's sorted values (device, B*k)
  OpDev *h_ops = nullptr;

  size_t *measure = nullptr;             // setup() only sums the device bytes it would take

  int setup(Workspace *hh, int B_, int64_t n_, int32_t k_, int32_t L_, int32_t m_, int32_t kind_,
            double tol_, uint64_t seed_, int32_t lz_steps_, bool mixed_ = false,
            bool var_deg_ = false, bool adaptive_ = false, bool mag_ = false) {
    mixed = mixed_;
    w_stale = true;
    var_deg = var_deg_;
    adaptive = adaptive_ && !var_deg_ && !mixed_;
    mag = mag_ && !mixed_ && !adaptive;
    m_base = m_;
    if (var_deg) m_ = kMaxDegree;          // coefficient tables sized for the largest degree
    if (adaptive) m_ = std::min(64, std::max(m_, 2 * m_));
    h = hh;
    st = hh->stream;
    B = B_;
    n = n_;
    k = k_;
    L = L_;
    m = m_;
    kind = kind_;
    tol = tol_;
    seed = seed_;
    lz_steps = lz_steps_;
    ld = round_up(n, 64);
    bs = ld * k;
    Nmax = 0;
    if (kind != SCSF_CSR) {               // square grids: side = sqrt(n), fixed for the engine
      Nmax = (int32_t)std::llround(std::sqrt((double)n));
      while ((int64_t)Nmax * Nmax < n) ++Nmax;
    }
    ldm = (int32_t)round_up(k, 32);
    part_stride = gemm_tn_partial_elems(n, ldm);
    const size_t blk = (size_t)B * bs;
    // every device buffer of the engine; with `measure` set only their sizes are summed (the
    // workspace query), and nothing is allocated or initialised
    auto alloc = [&](int id, size_t count, auto **out) -> int {
      using T = std::remove_pointer_t<std::remove_reference_t<decltype(out)>>;
      if (measure) {
        *measure += (std::max<size_t>(count * sizeof(*(*out)), 256) + 255) / 256 * 256;
        *out = nullptr;
        return SCSF_OK;
      }
      return grow(h, id, count, out);
    };
    STCHK(alloc(B_X, blk, &X));
    STCHK(alloc(B_Y1, blk, &Y1));
    STCHK(alloc(B_Y2, blk, &Y2));
    STCHK(alloc(B_W, blk, &W));
    STCHK(alloc(B_G, (size_t)B * ldm * ldm, &G));
    STCHK(alloc(B_M, (size_t)B * ldm * ldm, &M));
    STCHK(alloc(B_PART, (size_t)B * part_stride, &part));
    STCHK(alloc(B_THETA, (size_t)B * k, &theta));
    STCHK(alloc(B_RES, (size_t)B * k, &res));
    int32_t *ints = nullptr;
    STCHK(alloc(B_INT, (size_t)B * 7, &ints));
    lock = ints;
    nconv = ints + B;
    done = ints + 2 * B;
    flag = ints + 3 * B;
    need = ints + 4 * B;
    offv = ints + 5 * B;
    Lv = ints + 6 * B;
    STCHK(alloc(B_BND, (size_t)B * 4, &bnd));
    STCHK(alloc(B_COEF, (size_t)std::max(m, 1) * B * 3, &coef));
    if (mag) {
      STCHK(alloc(B_SQT, blk, &T));
      STCHK(alloc(B_SQP, blk, &P));
      STCHK(alloc(B_COEF2, (size_t)std::max(m, 1) * B * 3, &coef2));
    }
    STCHK(alloc(B_UNIT, (size_t)B * 3, &unit));
    STCHK(alloc(B_CHOL, (size_t)B * kMaxK * (kMaxK + 1), &chol));
    STCHK(alloc(B_JAC, (size_t)B * kMaxK * (kMaxK + 1), &jac));
    STCHK(alloc(B_REC, (size_t)B * jacobi_record_elems(k), &rec));
    STCHK(alloc(B_EIG, (size_t)B * tridiag_work_elems(k), &eigw));
    int32_t *rk = nullptr;
    STCHK(alloc(B_RANK, (size_t)B * ldm + B, &rk));
    ranks = rk;
    nsweeps = rk + (size_t)B * ldm;
    STCHK(alloc(B_LZ, (size_t)B * 3 * n, &lz));
    STCHK(alloc(B_OPS, (size_t)B, &ops));
    STCHK(alloc(B_HINT, (size_t)B * 3, &hint));
    STCHK(alloc(B_MDEG, (size_t)B, &mdeg));
    STCHK(alloc(B_ROWS, (size_t)B, &rows));
    STCHK(alloc(B_CDEG, (size_t)B * k, &cdeg));
    if (mixed) {
      float *e32 = nullptr;
      STCHK(alloc(B_E32, (size_t)3 * B * bs, &e32));
      if (e32) {
        E32[0] = e32;
        E32[1] = e32 + (size_t)B * bs;
        E32[2] = e32 + (size_t)2 * B * bs;
      }
      STCHK(alloc(B_R32, (size_t)B * bs, &R32));
      STCHK(alloc(B_SRC, (size_t)std::max(m, 1) * B * k, &src));
      STCHK(alloc(B_GAIN, (size_t)B * k, &gain));
      STCHK(alloc(B_WINB, (size_t)B * 3, &winb));
    }
    STCHK(alloc(B_SORTO, (size_t)B * k, &perm_d));   // extraction: column order, values
    STCHK(alloc(B_SORTV, (size_t)B * k, &vals_d));
    if (measure) return SCSF_OK;
    // pinned: 8 int arrays of B, perm B*k, theta/res/vals B*k, bnd B*4, unit B*3, ops B
    const size_t pin = (size_t)B * 11 * 4 + (size_t)B * k * 8 + (size_t)B * k * 24 +
                       (size_t)B * 4 * 8 + (size_t)B * 6 * 8 + (size_t)B * sizeof(OpDev) + 2048;
    STCHK(grow_pinned(h, pin));
    char *pp = static_cast<char *>(h->pinned);
    auto take = [&](size_t bytes) {
      char *r = pp;
      pp += (bytes + 63) / 64 * 64;
      return r;
    };
    // the int arrays in the device layout (lock | nconv | done | flag | need | off | L), so
    // the per-iteration readback and the state upload are one or two copies
    int32_t *h_ints = (int32_t *)take((size_t)B * 7 * 4);
    h_lock = h_ints;
    h_nconv = h_ints + B;
    h_done = h_ints + 2 * B;
    h_flag = h_ints + 3 * B;
    h_need = h_ints + 4 * B;
    h_off = h_ints + 5 * B;
    h_Lv = h_ints + 6 * B;
    h_perm = (int32_t *)take((size_t)B * k * 4);
    h_theta = (double *)take((size_t)B * k * 8);
    h_res = (double *)take((size_t)B * k * 8);
    h_vals = (double *)take((size_t)B * k * 8);
    h_bnd = (double *)take((size_t)B * 4 * 8);
    h_unit = (double *)take((size_t)B * 3 * 8);
    h_ops = (OpDev *)take((size_t)B * sizeof(OpDev));
    h_mdeg = (int32_t *)take(B * 4);
    h_mraw = (int32_t *)take(B * 4);
    h_rows = (int32_t *)take(B * 4);
    h_cdeg = (int32_t *)take((size_t)B * k * 4);
    h_hint = (double *)take((size_t)B * 3 * 8);
    if ((size_t)(pp - static_cast<char *>(h->pinned)) > h->pinned_bytes) return SCSF_ENOMEM;
    varw = false;
    for (int b = 0; b < B; ++b) {
      h_lock[b] = h_nconv[b] = h_done[b] = h_flag[b] = h_need[b] = h_off[b] = 0;
      h_Lv[b] = L;
      h_mdeg[b] = h_mraw[b] = adaptive ? m_base : m_;
      h_rows[b] = (int32_t)n;
      for (int c = 0; c < k; ++c) h_cdeg[(size_t)b * k + c] = m_base;
      h_hint[3 * b] = h_hint[3 * b + 1] = h_hint[3 * b + 2] = 0.0;
      h_unit[3 * b] = 1.0;
      h_unit[3 * b + 1] = 0.0;
      h_unit[3 * b + 2] = 0.0;
    }
    HIPCHK(hipMemcpyAsync(unit, h_unit, (size_t)B * 3 * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(hint, h_hint, (size_t)B * 3 * 8, hipMemcpyHostToDevice, st));
    // plan_degrees() uploads only when a degree differs from the mirror, so the device copy
    // must match the mirror from the start (the buffer is reused across calls)
    if (var_deg || adaptive)
      HIPCHK(hipMemcpyAsync(mdeg, h_mdeg, (size_t)B * 4, hipMemcpyHostToDevice, st));
    if (adaptive)
      HIPCHK(hipMemcpyAsync(cdeg, h_cdeg, (size_t)B * k * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(rows, h_rows, (size_t)B * 4, hipMemcpyHostToDevice, st));
    HIPCHK(fill_int(flag, 0, B, st));
    HIPCHK(hipStreamSynchronize(st));
    return make_events();
  }

  // Degrees of this iteration: the largest requested degree M over the unfinished problems;
  // every problem's degree is raised by at most 2 to the same residue mod 3 as M, so all
  // results end in the same buffer of the three-buffer ring.
  int plan_degrees() {
    int M = 1;
    for (int b = 0; b < B; ++b)
      if (!h_done[b]) M = std::max(M, h_mraw[b]);
    // every problem's filter must end in the buffer of the largest degree's: the three-buffer
    // ring needs equal residues mod 3, the fused groups (two buffer pairs in turn) mod 2 S
    const int mod = fused_filter(M) ? 2 * fuse : 3;
    bool changed = false;
    for (int b = 0; b < B; ++b) {
      int d = std::min(h_mraw[b], M);
      while ((M - d) % mod != 0) ++d;
      if (d != h_mdeg[b]) { h_mdeg[b] = d; changed = true; }
    }
    mcur = M;
    if (changed) {
      HIPCHK(hipMemcpyAsync(mdeg, h_mdeg, (size_t)B * 4, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    return SCSF_OK;
  }
  // Upload the hints of the listed slots only: the device marks a consumed hint (state 2/3),
  // and the other slots' host copies would still say "pending".
  int upload_hints(const std::vector<int> &slots) {
    for (int b : slots)
      HIPCHK(hipMemcpyAsync(hint + (size_t)b * 3, h_hint + (size_t)b * 3, 24,
                            hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCSF_OK;
  }

  // Uploads of the pinned mirrors complete before returning: the host edits the mirrors
  // again right after, and an asynchronous copy would read the edited values.
  int upload_state() {
    HIPCHK(hipMemcpyAsync(lock, h_lock, (size_t)B * 3 * 4, hipMemcpyHostToDevice, st));  // lock, nconv, done
    HIPCHK(hipMemcpyAsync(need, h_need, (size_t)B * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCSF_OK;
  }
  int upload_ops() {
    for (int b = 0; b < B; ++b) h_rows[b] = (int32_t)h_ops[b].n;
    HIPCHK(hipMemcpyAsync(ops, h_ops, (size_t)B * sizeof(OpDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(rows, h_rows, (size_t)B * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCSF_OK;
  }
  // per-slot widths k_b <= k and pair counts L_b < k_b (a mixed-width batch)
  int set_widths(const std::vector<int32_t> &kb, const std::vector<int32_t> &Lb) {
    varw = true;
    for (int b = 0; b < B; ++b) {
      h_off[b] = k - kb[b];
      h_Lv[b] = Lb[b];
      h_lock[b] = h_nconv[b] = h_off[b];
    }
    HIPCHK(hipMemcpyAsync(offv, h_off, (size_t)B * 2 * 4, hipMemcpyHostToDevice, st));  // off, L
    HIPCHK(hipStreamSynchronize(st));
    return SCSF_OK;
  }
  int download_state() {
    HIPCHK(hipMemcpyAsync(h_lock, lock, (size_t)B * 4 * 4, hipMemcpyDeviceToHost, st));  // lock..flag
    if (adaptive) {
      HIPCHK(hipMemcpyAsync(h_mdeg, mdeg, (size_t)B * 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(h_cdeg, cdeg, (size_t)B * k * 4, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    prof_drain(h);
    return SCSF_OK;
  }
  // a reloaded problem starts its adaptive degrees again from the configured degree
  int reset_degrees(const std::vector<int> &slots) {
    if (!adaptive) return SCSF_OK;
    for (int b : slots) {
      HIPCHK(fill_int(cdeg + (size_t)b * k, m_base, k, st));
      HIPCHK(fill_int(mdeg + b, m_base, 1, st));
      h_mdeg[b] = m_base;
      for (int c = 0; c < k; ++c) h_cdeg[(size_t)b * k + c] = m_base;
    }
    return SCSF_OK;
  }

  // Algorithmic HBM bytes of one filter step: each active column of the input block (and of
  // the previous block after the first step) read once, the output written once, and the
  // operator coefficients read once per problem (5-point: the two face arrays plus the
  // potential when present; 9-point: one cell tensor).  Rows are per problem.
  double step_bytes(bool has_prev, bool fp32 = false, int step = 0) const {
    double vec = 0.0, coeff = 0.0;
    for (int b = 0; b < B; ++b)
      if (!h_done[b] && (!var_deg || step < h_mdeg[b])) {
        const double nb = (double)h_rows[b];
        int cols = k - h_lock[b];
        if (adaptive) {                     // columns still inside their degree at this step
          cols = 0;
          for (int c = h_lock[b]; c < k; ++c) {
            int32_t d = h_cdeg[(size_t)b * k + c];
            d += ((mcur - d) % 3 + 3) % 3;
            cols += step < d;
          }
          if (cols == 0) continue;
        }
        vec += nb * (double)cols;
        coeff += (kind == SCSF_STENCIL5) ? (h_ops[b].v ? 3.0 : 2.0) * nb
                 : (kind == SCSF_STENCIL9 || kind == SCSF_PLATE) ? (kind == SCSF_PLATE ? 2.0 : 3.0) * nb
                 : 0.0;
      }
    if (fp32)  // e_i, e_{i-1}, r read, e_{i+1} written in FP32
      return 4.0 * (has_prev ? 4.0 : 3.0) * vec + 8.0 * coeff;
    return 8.0 * ((has_prev ? 3.0 : 2.0) * vec + coeff);
  }

  // upper bounds of the problems with h_need[b] set
  // the same from a table computed up front for every operator of the call (host, 4 doubles
  // per operator, indexed by opid[b]): only the rows of the problems with h_need[b] set move
  int set_bounds(const double *table, const int32_t *opid) {
    HIPCHK(hipEventRecord(pev[5], st));
    for (int b = 0; b < B; ++b) {
      if (!h_need[b]) continue;
      std::copy(table + (size_t)opid[b] * 4, table + (size_t)opid[b] * 4 + 4, h_bnd + (size_t)b * 4);
      HIPCHK(hipMemcpyAsync(bnd + (size_t)b * 4, h_bnd + (size_t)b * 4, 32, hipMemcpyHostToDevice,
                            st));
    }
    HIPCHK(hipEventRecord(pev[6], st));
    HIPCHK(hipEventSynchronize(pev[6]));
    std::vector<char> who(B);
    for (int b = 0; b < B; ++b) who[b] = h_need[b] != 0;
    charge(PH_BOUND, span(5, 6), who);
    return SCSF_OK;
  }
  int compute_bounds() {
    HIPCHK(hipEventRecord(pev[5], st));
    HIPCHK(bounds(ops, B, kind, n, lz_steps, seed ^ 0x5DEECE66DULL, need, lz, bnd, st, mag));
    HIPCHK(hipEventRecord(pev[6], st));
    HIPCHK(hipEventSynchronize(pev[6]));
    std::vector<char> who(B);
    for (int b = 0; b < B; ++b) who[b] = h_need[b] != 0;
    charge(PH_BOUND, span(5, 6), who);
    return SCSF_OK;
  }

  // X active columns <- orthonormal basis (block Gram-Schmidt twice against the locked
  // columns, then CholeskyQR2, with a third pass for problems that needed the shift)
  int orth(double *Yf, bool cgs) {
    if (cgs) {
      for (int rep = 0; rep < 2; ++rep) {
        HIPCHK(gemm_tn(B, n, ld, X, bs, COLS_LOCKED, Yf, bs, COLS_ACTIVE, k, lock, false, part,
                       part_stride, G, ldm, nullptr, 0, st, rows));
        HIPCHK(gemm_nn(B, n, ld, X, bs, COLS_LOCKED, Yf, bs, COLS_ACTIVE, k, lock, G, ldm, -1.0,
                       1.0, nullptr, 0, nullptr, 0, st, rows));
      }
    }
    for (int pass = 0; pass < 3; ++pass) {
      const int32_t *gate = (pass == 2) ? flag : nullptr;
      HIPCHK(gemm_tn(B, n, ld, Yf, bs, COLS_ACTIVE, Yf, bs, COLS_ACTIVE, k, lock, true, part,
                     part_stride, G, ldm, gate, 4, st, rows));
      HIPCHK(chol_inv(B, n, k, lock, G, M, ldm, flag, gate, 4, chol, st));
      HIPCHK(gemm_nn(B, n, ld, Yf, bs, COLS_ACTIVE, Yf, bs, COLS_ACTIVE, k, lock, M, ldm, 1.0, 0.0,
                     gate, 4, flag, 3, st, rows));
    }
    return SCSF_OK;
  }

  // Rayleigh-Ritz on the orthonormal active columns of Yf; Ritz vectors land in X, A X in W
  // Jacobi accuracy for the convergence target: an off-diagonal entry delta sqrt|g_pp g_qq|
  // left in G moves a Ritz vector's relative residual by about delta sqrt(theta_i / theta_j),
  // so delta = tol / 100 keeps it well below tol (bounded to [1e-14, 1e-10]).
  double jacobi_stop() const { return std::min(1e-10, std::max(1e-14, 0.01 * tol)); }
  int rayleigh_ritz(double *Yf) {
    HIPCHK(spmm_step(ops, B, kind, n, Nmax, Yf, nullptr, W, ld, bs, COLS_ACTIVE, k, lock, unit, false,
                     st, nullptr, 0, cpt, pot));
    HIPCHK(gemm_tn(B, n, ld, Yf, bs, COLS_ACTIVE, W, bs, COLS_ACTIVE, k, lock, true, part,
                   part_stride, G, ldm, nullptr, 0, st, rows));
    if (eig == SCSF_EIG_JACOBI)
      HIPCHK(jacobi_eig(B, k, lock, G, M, ldm, theta, flag, jac, rec, ranks, nsweeps, st,
                        jacobi_stop()));
    else
      HIPCHK(tridiag_eig(B, k, lock, G, M, ldm, theta, flag, jac, eigw, st));
    double *Zr = M;
    if (mag) {                        // pairs by |theta|; the Gram buffer takes the reordered Z
      HIPCHK(magnitude_order(B, k, lock, theta, M, G, ldm, st));
      Zr = G;
    }
    HIPCHK(gemm_nn(B, n, ld, Yf, bs, COLS_ACTIVE, X, bs, COLS_ACTIVE, k, lock, Zr, ldm, 1.0, 0.0,
                   nullptr, 0, nullptr, 0, st, rows));
    HIPCHK(gemm_nn(B, n, ld, W, bs, COLS_ACTIVE, W, bs, COLS_ACTIVE, k, lock, Zr, ldm, 1.0, 0.0,
                   nullptr, 0, nullptr, 0, st, rows));
    return SCSF_OK;
  }

  // Cold start of the listed problems while every other problem is parked (lock = k):
  // Gaussian block (on the problem's own columns; the placeholders below off_b are zeroed),
  // orthonormalisation and one Rayleigh-Ritz (no locking).
  int cold_start(const std::vector<int> &slots) {
    std::vector<int32_t> saved(h_lock, h_lock + B);
    for (int b = 0; b < B; ++b) h_lock[b] = k;
    for (int b : slots) {
      const int o = off(b);
      h_lock[b] = o;
      HIPCHK(zero_columns(ld, o, X + (int64_t)b * bs, ld, st));
      HIPCHK(gaussian_fill(1, h_rows[b], ld, bs, k - o, X + (int64_t)b * bs + (int64_t)o * ld,
                           seed * 0x9E3779B97F4A7C15ULL + (uint64_t)b * 0xD1B54A32D192ED03ULL + 1,
                           st));
    }
    STCHK(upload_state());
    HIPCHK(fill_int(flag, 0, B, st));
    HIPCHK(hipEventRecord(pev[5], st));
    STCHK(orth(X, false));
    HIPCHK(hipEventRecord(pev[6], st));
    STCHK(rayleigh_ritz(X));
    HIPCHK(hipEventRecord(pev[7], st));
    for (int b = 0; b < B; ++b) h_lock[b] = saved[b];
    for (int b : slots) h_lock[b] = off(b);
    STCHK(upload_state());
    std::vector<char> who(B, 0);
    for (int b : slots) who[b] = 1;
    charge(PH_ORTH, span(5, 6), who);
    charge(PH_RR, span(6, 7), who);
    return SCSF_OK;
  }

  std::vector<int32_t> lock_before;
  int32_t h_lock_prev(int b) const { return lock_before.empty() ? off(b) : lock_before[b]; }

  // The three parts of one outer iteration: window + coefficients, the degree-M filter, and
  // orthonormalisation + Rayleigh-Ritz + residuals + locking.  All of them only launch
  // kernels on `st`, so each can be captured into a graph and replayed.
  int enqueue_pre(int M) {
    HIPCHK(fill_int(flag, 0, B, st));
    HIPCHK(cheb_coeffs(B, k, M, theta, bnd, done, coef, mixed ? winb : nullptr, hint, st,
                       mag ? coef2 : nullptr, varw ? offv : nullptr));
    return SCSF_OK;
  }
  int enqueue_filter(int M, bool timed) {
    const int32_t *md = var_deg ? mdeg : nullptr;   // adaptive degrees are per column (cdeg)
    if (mixed) {
      // Y = p_m(A) X = X p_m(Theta) + e_m with the correction e in FP32 (misc.hip)
      HIPCHK(mp_tables(B, k, M, theta, winb, lock, done, src, gain, md, st));
      HIPCHK(mp_prep(B, n, ld, bs, k, lock, X, W, theta, coef, R32, E32[1], st));
      for (int s = 1; s < M; ++s) {
        const int slot = timed ? prof_begin(h, step_bytes(s > 1, true, s)) : -1;
        HIPCHK(spmm_step32(ops, B, kind, n, Nmax, E32[s % 3], E32[(s + 2) % 3], E32[(s + 1) % 3], ld, bs,
                           COLS_ACTIVE, k, lock, coef + (size_t)s * B * 3, s > 1, R32,
                           src + (size_t)s * B * k, st, md, s, cpt, pot));
        prof_end(h, slot);
      }
      HIPCHK(mp_final(B, n, ld, bs, k, lock, X, E32[M % 3], gain, Y1, st));
    } else if (mag) {
      // Y_{s+1} = a A (A Y_s) + b Y_s + g Y_{s-1}: T = A Y_s, P = b Y_s + g Y_{s-1}, then the
      // step kernel with (a, 0, 1) on (T, P)
      double *ring[3] = {X, Y1, Y2};
      for (int s = 0; s < M; ++s) {
        HIPCHK(spmm_step(ops, B, kind, n, Nmax, ring[s % 3], nullptr, T, ld, bs, COLS_ACTIVE, k,
                         lock, unit, false, st, nullptr, s, cpt, pot));
        HIPCHK(axpby_active(B, n, ld, bs, k, lock, ring[s % 3], s > 0 ? ring[(s + 2) % 3] : nullptr,
                            coef + (size_t)s * B * 3, P, rows, st));
        HIPCHK(spmm_step(ops, B, kind, n, Nmax, T, P, ring[(s + 1) % 3], ld, bs, COLS_ACTIVE, k,
                         lock, coef2 + (size_t)s * B * 3, true, st, nullptr, s, cpt, pot));
      }
    } else if (fused_filter(M)) {
      // q = M mod S single steps in the three-buffer ring, then groups of S steps, each from
      // the two newest levels in one pair of buffers to the next two in the other pair
      const int q = M % fuse;
      double *ring[3] = {X, Y1, Y2};
      for (int s = 0; s < q; ++s) {
        const int slot = timed ? prof_begin(h, step_bytes(s > 0, false, s)) : -1;
        HIPCHK(spmm_step(ops, B, kind, n, Nmax, ring[s % 3], ring[(s + 2) % 3], ring[(s + 1) % 3],
                         ld, bs, COLS_ACTIVE, k, lock, coef + (size_t)s * B * 3, s > 0, st, md,
                         s, cpt, pot, nullptr, M));
        prof_end(h, slot);
      }
      FusedPlan fp = fused_plan(M);
      double *cur = fp.in_cur, *prv = fp.in_prv;
      for (int g = 0, s0 = q; s0 < M; ++g, s0 += fuse) {
        double *oc = (g & 1) ? fp.odd_cur : fp.even_cur;
        double *op = (g & 1) ? fp.odd_prv : fp.even_prv;
        double bytes = 0.0;
        if (timed)
          for (int s = s0; s < s0 + fuse; ++s) bytes += step_bytes(s > 0, false, s);
        const int slot = timed ? prof_begin(h, bytes, fuse) : -1;
        HIPCHK(spmm_fused(ops, B, kind, n, Nmax, cur, s0 > 0 ? prv : nullptr, oc, op, ld, bs,
                          COLS_ACTIVE, k, lock, coef + (size_t)s0 * B * 3, fuse, st, md, s0,
                          cpt, pot));
        prof_end(h, slot);
        cur = oc;
        prv = op;
      }
    } else {
      double *ring[3] = {X, Y1, Y2};
      for (int s = 0; s < M; ++s) {
        const int slot = timed ? prof_begin(h, step_bytes(s > 0, false, s)) : -1;
        HIPCHK(spmm_step(ops, B, kind, n, Nmax, ring[s % 3], ring[(s + 2) % 3], ring[(s + 1) % 3],
                         ld, bs, COLS_ACTIVE, k, lock, coef + (size_t)s * B * 3, s > 0, st, md,
                         s, cpt, pot, adaptive ? cdeg : nullptr, M));
        prof_end(h, slot);
      }
    }
    return SCSF_OK;
  }
  // The fused filter runs for the plain FP64 filter of the grid stencils when the degree
  // holds at least one group.
  bool fused_filter(int M) const {
    return fuse >= 2 && M >= fuse && !mixed && !mag && !adaptive &&
           spmm_fused_supported(kind, Nmax, fuse);
  }
  // Buffers of the fused schedule of degree M: after the q = M mod S single steps the two
  // newest levels are in (in_cur, in_prv) (X alone when q = 0); the groups write to the two
  // other buffers, then back, in turn.  In each pair the newest level goes to the buffer that
  // is not W (the Rayleigh-Ritz step writes A Q into W), so the filtered block never is W.
  struct FusedPlan {
    double *in_cur, *in_prv, *even_cur, *even_prv, *odd_cur, *odd_prv;
  };
  FusedPlan fused_plan(int M) const {
    const int q = M % fuse;
    double *ring[3] = {X, Y1, Y2};
    FusedPlan fp{};
    fp.in_cur = ring[q % 3];
    fp.in_prv = q > 0 ? ring[(q + 2) % 3] : nullptr;
    double *all[4] = {X, Y1, Y2, W};
    double *other[4];
    int no = 0;
    for (double *p : all)
      if (p != fp.in_cur && p != fp.in_prv) other[no++] = p;
    // q = 0: three buffers are free; the first group's pair takes Y1, Y2 and the second X, W
    double *e0 = other[0], *e1 = other[1];
    if (q == 0) { e0 = Y1; e1 = Y2; }
    auto order = [&](double *a, double *b2, double **c, double **pv) {
      if (a == W) std::swap(a, b2);
      *c = a;
      *pv = b2;
    };
    order(e0, e1, &fp.even_cur, &fp.even_prv);
    double *o0 = fp.in_cur, *o1 = fp.in_prv;
    if (q == 0) { o0 = X; o1 = W; }
    order(o0, o1, &fp.odd_cur, &fp.odd_prv);
    return fp;
  }
  double *filtered(int M) const {
    double *ring[3] = {X, Y1, Y2};
    if (mixed) return Y1;
    if (fused_filter(M)) {
      const int groups = (M - M % fuse) / fuse;
      const FusedPlan fp = fused_plan(M);
      return (groups & 1) ? fp.even_cur : fp.odd_cur;
    }
    return ring[M % 3];
  }
  int enqueue_orth(int M) { return orth(filtered(M), true); }
  int enqueue_rr(int M) { return rayleigh_ritz(filtered(M)); }
  int enqueue_post(int /*M*/) {
    HIPCHK(residuals(B, n, ld, X, W, bs, k, lock, theta, res, st, rows));
    HIPCHK(lock_update(B, k, L, tol, lock, nconv, res, theta, mag ? 1 : mag_low ? 2 : 0, done,
                       flag, st, varw ? offv : nullptr, varw ? Lv : nullptr));
    if (adaptive)
      HIPCHK(adaptive_degrees(B, k, lock, done, theta, res, bnd, tol, m_base, m, cdeg, mdeg, st));
    return SCSF_OK;
  }

  // Graphs of the five parts, one set per filter degree (the only launch parameter that
  // changes between iterations; every kernel reads its per-problem state from device memory).
  struct GraphSet {
    int M = 0;
    hipGraphExec_t pre = nullptr, filt = nullptr, orth = nullptr, rr = nullptr, post = nullptr;
  };
  bool use_graph = false;
  std::vector<GraphSet> gcache;
  static constexpr int kMaxGraphSets = 16;

  template <typename F>
  int capture(F &&body, hipGraphExec_t *out) {
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != SCSF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(e);
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ei);
    return SCSF_OK;
  }
  static void drop_set(GraphSet &gs) {
    for (hipGraphExec_t *g : {&gs.pre, &gs.filt, &gs.orth, &gs.rr, &gs.post})
      if (*g) {
        (void)hipGraphExecDestroy(*g);
        *g = nullptr;
      }
  }
  void drop_graphs() {
    for (auto &gs : gcache) drop_set(gs);
    gcache.clear();
  }
  int graphs_for(int M, GraphSet **out) {
    for (auto &gs : gcache)
      if (gs.M == M) { *out = &gs; return SCSF_OK; }
    if ((int)gcache.size() >= kMaxGraphSets) {
      HIPCHK(hipStreamSynchronize(st));
      drop_graphs();
    }
    GraphSet gs;
    gs.M = M;
    int rc = capture([&] { return enqueue_pre(M); }, &gs.pre);
    if (rc == SCSF_OK) rc = capture([&] { return enqueue_filter(M, false); }, &gs.filt);
    if (rc == SCSF_OK) rc = capture([&] { return enqueue_orth(M); }, &gs.orth);
    if (rc == SCSF_OK) rc = capture([&] { return enqueue_rr(M); }, &gs.rr);
    if (rc == SCSF_OK) rc = capture([&] { return enqueue_post(M); }, &gs.post);
    if (rc != SCSF_OK) {
      drop_set(gs);
      return rc;
    }
    gcache.push_back(gs);
    *out = &gcache.back();
    return SCSF_OK;
  }

  Engine() = default;
  Engine(const Engine &) = delete;
  Engine &operator=(const Engine &) = delete;
  ~Engine() {
    if (!gcache.empty()) {
      (void)hipStreamSynchronize(st);
      drop_graphs();
    }
    for (hipEvent_t &ev : pev)
      if (ev) (void)hipEventDestroy(ev);
  }

  // Per-phase device times: events on the lane's stream at the phase boundaries, read after
  // the synchronisation that follows them.  ph[b] accumulates the times of the launches
  // problem b took part in (shared with the other problems of the batch).
  hipEvent_t pev[8] = {};                  // 0-4 outer iteration, 5-6 bounds, 5-7 cold start
  std::vector<std::array<double, PH_COUNT>> ph;
  int make_events() {
    for (hipEvent_t &ev : pev)
      if (!ev) HIPCHK(hipEventCreate(&ev));
    ph.assign(B, std::array<double, PH_COUNT>{});
    return SCSF_OK;
  }
  float span(int a, int b) const {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, pev[a], pev[b]) == hipSuccess ? ms : 0.f;
  }
  void charge(int phase, float ms, const std::vector<char> &who) {
    h->phase_ms[phase] += ms;
    for (int b = 0; b < B; ++b)
      if (who[b]) ph[b][phase] += ms;
  }

  // One outer iteration of Algorithm 3 for every problem not done.
  int iterate() {
    lock_before.assign(h_nconv, h_nconv + B);
    int M = m;
    if (var_deg) {
      STCHK(plan_degrees());
      M = mcur;
    } else if (adaptive) {                // the largest column degree of the unfinished problems
      M = m_base;
      for (int b = 0; b < B; ++b)
        if (!h_done[b]) M = std::max(M, std::min<int32_t>(h_mdeg[b], m));
      mcur = M;
      it_cols.assign(B, 0);
      it_deg.assign(B, 0);
      for (int b = 0; b < B; ++b) {
        if (h_done[b]) continue;
        for (int c = h_lock[b]; c < k; ++c) {
          int32_t d = h_cdeg[(size_t)b * k + c];
          d += ((M - d) % 3 + 3) % 3;
          it_cols[b] += d;
          it_deg[b] = std::max(it_deg[b], d);
        }
      }
    }
    std::vector<char> act(B);
    for (int b = 0; b < B; ++b) act[b] = !h_done[b];
    GraphSet *gs = nullptr;
    if (use_graph) STCHK(graphs_for(M, &gs));
    HIPCHK(hipEventRecord(pev[0], st));
    if (mixed && w_stale) {           // A X of newly loaded operators (residual form)
      HIPCHK(spmm_step(ops, B, kind, n, Nmax, X, nullptr, W, ld, bs, COLS_ACTIVE, k, lock, unit,
                       false, st, nullptr, 0, cpt, pot));
      w_stale = false;
    }
    if (!use_graph) {
      STCHK(enqueue_pre(M));
      STCHK(enqueue_filter(M, h->prof && !mag));
      HIPCHK(hipEventRecord(pev[1], st));
      STCHK(enqueue_orth(M));
      HIPCHK(hipEventRecord(pev[2], st));
      STCHK(enqueue_rr(M));
      HIPCHK(hipEventRecord(pev[3], st));
      STCHK(enqueue_post(M));
    } else {
      HIPCHK(hipGraphLaunch(gs->pre, st));
      int slot = -1;
      if (h->prof && !mag) {          // one timed span over the filter graph's M launches
        double bytes = 0.0;
        for (int s = mixed ? 1 : 0; s < M; ++s)
          bytes += mixed ? step_bytes(s > 1, true, s) : step_bytes(s > 0, false, s);
        slot = prof_begin(h, bytes, mixed ? M - 1 : M);
      }
      HIPCHK(hipGraphLaunch(gs->filt, st));
      prof_end(h, slot);
      HIPCHK(hipEventRecord(pev[1], st));
      HIPCHK(hipGraphLaunch(gs->orth, st));
      HIPCHK(hipEventRecord(pev[2], st));
      HIPCHK(hipGraphLaunch(gs->rr, st));
      HIPCHK(hipEventRecord(pev[3], st));
      HIPCHK(hipGraphLaunch(gs->post, st));
    }
    HIPCHK(hipEventRecord(pev[4], st));
    STCHK(download_state());
    charge(PH_FILTER, span(0, 1), act);
    charge(PH_ORTH, span(1, 2), act);
    charge(PH_RR, span(2, 3), act);
    charge(PH_RESID, span(3, 4), act);
    return SCSF_OK;
  }

  // theta / res / bnd / hint of every slot to the pinned mirrors (four copies and one wait
  // for all the problems that finished in an iteration; the host reads only those slots)
  int fetch(const std::vector<int> &slots) {
    if (slots.empty()) return SCSF_OK;
    HIPCHK(hipMemcpyAsync(h_theta, theta, (size_t)B * k * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_res, res, (size_t)B * k * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_bnd, bnd, (size_t)B * 4 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_hint, hint, (size_t)B * 3 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return SCSF_OK;
  }
  int fetch(int b) { return fetch(std::vector<int>{b}); }

  // The L smallest converged pairs of problem b (of its first max(L, nconv) columns: a
  // solve that ends converged may hold more than L, and a pair that entered the block late
  // is locked after larger ones), ascending -> evals (device, L) and evecs (device, n x L,
  // ld ldo), canonical sign.  Needs fetch(b) first.  Returns max relative residual of the
  // pairs.
  // With mag_low: the L of the lowest converged pairs smallest in |theta|, in that order, and
  // *certified = false when the block ran out of pairs before the certificate held.
  int prepare_extract(int b, double *maxres, bool *certified = nullptr) {
    // the problem's own columns [o, k) and pair count (per-slot widths; else 0 and L)
    const int o = off(b), Lb = Lof(b), kb = k - o;
    const double *th = h_theta + (size_t)b * k + o;
    int32_t *perm = h_perm + (size_t)b * k;
    const int nc = std::min<int>(h_nconv[b] - o, kb);
    int nsel = std::max<int>(Lb, nc);
    std::iota(perm, perm + nsel, 0);
    if (mag_low) {
      // the lowest converged pairs (at or below the smallest unconverged Ritz value), ordered
      // by |theta|; their first L are the wanted ones when the certificate held
      const double tu = nc < kb ? th[nc] : INFINITY;
      int q = 0;
      for (int c = 0; c < nc; ++c)
        if (th[c] <= tu) perm[q++] = c;
      if (q >= Lb) {
        nsel = q;
      } else {
        nsel = std::max<int>(Lb, nc);
        std::iota(perm, perm + nsel, 0);
      }
      std::stable_sort(perm, perm + nsel,
                       [&](int a, int c) { return std::fabs(th[a]) < std::fabs(th[c]); });
    } else if (mag) {
      std::stable_sort(perm, perm + nsel,
                       [&](int a, int c) { return std::fabs(th[a]) < std::fabs(th[c]); });
    } else {
      std::stable_sort(perm, perm + nsel, [&](int a, int c) { return th[a] < th[c]; });
    }
    // a lower end that gave up (flag bit 16) or ran out of iterations is not certified
    if (certified) *certified = !(mag_low && ((h_flag[b] & 16) || !h_done[b]));
    double *vals = h_vals + (size_t)b * k;
    double mr = 0.0;
    for (int j = 0; j < Lb; ++j) mr = std::max(mr, h_res[(size_t)b * k + o + perm[j]]);
    for (int j = 0; j < Lb; ++j) vals[j] = th[perm[j]];
    if (maxres) *maxres = mr;
    return SCSF_OK;
  }
  // The column orders and sorted values of every slot to the device, one copy each (for the
  // slots prepared since the last fetch: the host writes these rows again only after the
  // next fetch, which waits for the stream).
  int upload_extract() {
    HIPCHK(hipMemcpyAsync(perm_d, h_perm, (size_t)B * k * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(vals_d, h_vals, (size_t)B * k * 8, hipMemcpyHostToDevice, st));
    return SCSF_OK;
  }
  // evals (device, L) and evecs (device, n x L, ld ldo) of slot b, canonical sign, from its
  // prepared and uploaded order; no wait (the caller's solve returns after its streams)
  int launch_extract(int b, double *evals, double *evecs, int64_t ldo) {
    const int o = off(b), Lb = Lof(b);
    HIPCHK(gather_columns_signed(h_rows[b], Lb, X + (int64_t)b * bs + (int64_t)o * ld, ld,
                                 perm_d + (size_t)b * k, evecs, ldo, st, vals_d + (size_t)b * k,
                                 evals));
    if (h_ops[b].kind == SCSF_PLATE)             // u = M^{-1/2} y, M-orthonormal
      HIPCHK(scale_rows_rsqrt(h_rows[b], Lb, evecs, ldo, h_ops[b].wy, st));
    return SCSF_OK;
  }
  // one problem: prepare, upload and launch
  int extract(int b, double *evals, double *evecs, int64_t ldo, double *maxres,
              bool *certified = nullptr) {
    STCHK(prepare_extract(b, maxres, certified));
    STCHK(upload_extract());
    return launch_extract(b, evals, evecs, ldo);
  }
};

// status of a finished (or abandoned) solve from its flags
int solve_status(int32_t flagv, bool converged) {
  if (flagv & 2) return SCSF_ENUMERIC;
  if (flagv & 1) return SCSF_EBREAKDOWN;
  return converged ? SCSF_OK : SCSF_ENOTCONV;
}

int check_params(const scsf_params *p, int64_t n) {
  if (!p) return SCSF_EINVAL;
  if (p->L <= 0 || p->k <= p->L || p->k > kMaxK || p->k > n) return SCSF_EINVAL;
  if (p->degree < 1 || p->degree > kMaxDegree) return SCSF_EINVAL;
  if (p->precision == SCSF_MIXED && p->degree > kMaxDegreeMixed) return SCSF_EINVAL;
  if (!(p->tol > 0.0)) return SCSF_EINVAL;
  if (p->lanczos_steps < 0 || p->lanczos_steps > 128) return SCSF_EINVAL;
  if (p->precision != SCSF_FP64 && p->precision != SCSF_MIXED) return SCSF_EINVAL;
  if (p->schedule != SCSF_SCHED_STATIC && p->schedule != SCSF_SCHED_DYNAMIC) return SCSF_EINVAL;
  if (p->adaptive != 0 && p->adaptive != 1) return SCSF_EINVAL;
  if (p->adaptive && p->precision != SCSF_FP64) return SCSF_EINVAL;
  if (p->cold_start != 0 && p->cold_start != 1) return SCSF_EINVAL;
  if (p->target != SCSF_TARGET_SMALLEST && p->target != SCSF_TARGET_MAGNITUDE) return SCSF_EINVAL;
  if (p->target == SCSF_TARGET_MAGNITUDE && (p->precision != SCSF_FP64 || p->adaptive))
    return SCSF_EINVAL;
  return SCSF_OK;
}

// The chained solve of a set of chunks on one workspace (one lockstep batch, one stream):
// chunk c covers order_host[cb[c] .. ce[c]).
// With `next` (dynamic schedule) a chain that finishes an operator takes order position
// next->fetch_add(1) instead of the next position of its own chunk; cb holds the chains' first
// positions and ce is ignored.
// One group of an uneven batch: operators sharing (kind, L, k), with sizes up to nmax, whose
// outputs sit at per-operator offsets of packed arrays.
struct Group {
  int32_t L = 0, k = 0;
  int64_t nmax = 0;
  const int64_t *eoff = nullptr, *voff = nullptr;   // evals / evecs offsets by operator index
};

// The chains of one lockstep batch over several (L, k) groups: per chain, its group's width
// and pair count and, with the dynamic schedule, its group's counter and the end of its
// group's range in the order (the groups' orders are concatenated).  The batch's block width
// is the largest k.
struct Mix {
  std::vector<int32_t> L, k;
  std::vector<std::atomic<int> *> next;   // null entries: static schedule
  std::vector<int32_t> end;
};

// Grid stencils on square grids: the Ritz vectors can move between sides by interpolation.
bool on_square_grid(const OpDev &o) {
  return (o.kind == SCSF_STENCIL5 || o.kind == SCSF_STENCIL9 || o.kind == SCSF_PLATE) &&
         (int64_t)o.N * o.N == o.n;
}

// Spectral bounds (Gershgorin + Lanczos, the engine's window bound) of every operator of a
// chained solve, computed up front in batched launches (one workgroup per operator) instead of
// one problem at a time when a lane loads it.  The Lanczos start vector is keyed by the
// operator's index, so an operator's bound does not depend on the schedule.  Returns the
// table on the host (4 doubles per operator, operator index order).
constexpr int kPreBoundBatch = 256;
size_t prebound_bytes(int32_t n_op, int64_t nmax) {
  auto a = [](size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; };
  const size_t batch = std::min<int32_t>(n_op, kPreBoundBatch);
  return a((size_t)n_op * sizeof(OpDev)) + a(batch * 3 * (size_t)nmax * 8) +
         a((size_t)n_op * 4 * 8);
}
int prebound(Workspace *w, const scsf_operator *ops_host, int32_t n_op, int32_t steps,
             uint64_t seed, std::vector<double> &table) {
  int64_t nmax = 0;
  for (int i = 0; i < n_op; ++i) nmax = std::max(nmax, ops_host[i].n);
  const int batch = std::min<int32_t>(n_op, kPreBoundBatch);
  OpDev *ops_d = nullptr;
  double *work = nullptr, *tab = nullptr;
  STCHK(grow(w, B_PREOPS, (size_t)n_op, &ops_d));
  STCHK(grow(w, B_PRELZ, (size_t)batch * 3 * nmax, &work));
  STCHK(grow(w, B_PREBND, (size_t)n_op * 4, &tab));
  std::vector<OpDev> h(n_op);
  for (int i = 0; i < n_op; ++i) h[i] = to_dev(ops_host[i]);
  HIPCHK(hipMemcpyAsync(ops_d, h.data(), (size_t)n_op * sizeof(OpDev), hipMemcpyHostToDevice,
                        w->stream));
  for (int i0 = 0; i0 < n_op; i0 += batch)
    HIPCHK(bounds(ops_d + i0, std::min(batch, n_op - i0), ops_host[0].kind, nmax, steps,
                  seed ^ 0x5DEECE66DULL, nullptr, work, tab + (size_t)i0 * 4, w->stream, false,
                  (uint32_t)i0));
  table.resize((size_t)n_op * 4);
  HIPCHK(hipMemcpyAsync(table.data(), tab, (size_t)n_op * 4 * 8, hipMemcpyDeviceToHost,
                        w->stream));
  HIPCHK(hipStreamSynchronize(w->stream));
  return SCSF_OK;
}

// Operators of a smallest-magnitude solve whose lower-end result could not be certified; the
// lanes add to it concurrently, and the caller solves them again with the squared filter.
struct Fallback {
  std::mutex mu;
  std::vector<int32_t> ops;
  void add(int32_t o) {
    std::lock_guard<std::mutex> lk(mu);
    ops.push_back(o);
  }
};

// How a SCSF_TARGET_MAGNITUDE solve runs: from the lower end of the spectrum first (lock
// kernel mode 2), with the squared filter when that could not be certified.
bool magnitude_lower_end(const scsf_params *prm, bool square_forced) {
  return prm->target == SCSF_TARGET_MAGNITUDE && !square_forced;
}

int run_chains(Workspace *w, const scsf_operator *ops_host, const int32_t *order_host,
               int32_t n_op, const std::vector<int> &cb, const std::vector<int> &ce,
               std::atomic<int> *next, const scsf_params *prm, const double *hints_host,
               double *evals, double *evecs, double *ritz, scsf_stats *stats_host,
               const Group *grp = nullptr, bool graphs = false, int cpt = 4,
               int eig = SCSF_EIG_JACOBI, Fallback *fallback = nullptr,
               bool square_forced = false, int fuse = 0, const double *bnd_table = nullptr,
               const Mix *mix = nullptr) {
  const int chains = (int)cb.size();
  if (chains == 0) return SCSF_OK;
  const int64_t n = grp ? grp->nmax : ops_host[0].n;
  const int32_t kind = ops_host[order_host[0]].kind;
  const int max_iter = prm->max_iter > 0 ? prm->max_iter : 5000;
  const int lzs = prm->lanczos_steps > 0 ? prm->lanczos_steps : 20;
  const int32_t L = grp ? grp->L : prm->L, k = grp ? grp->k : prm->k, m = prm->degree;
  const int64_t *eoff = grp ? grp->eoff : nullptr, *voff = grp ? grp->voff : nullptr;
  const bool low = magnitude_lower_end(prm, square_forced);
  const bool square = prm->target == SCSF_TARGET_MAGNITUDE && !low;

  Engine e;
  STCHK(e.setup(w, chains, n, k, L, m, kind, prm->tol, prm->seed, lzs,
                prm->precision == SCSF_MIXED, hints_host != nullptr, prm->adaptive != 0,
                square));
  e.mag_low = low;
  e.use_graph = graphs && w->own_stream;     // capture needs a stream of our own
  e.cpt = cpt;
  e.eig = eig;
  e.fuse = fuse;
  e.pot = false;                             // fixed for the engine: graphs keep the choice
  for (int i = 0; i < n_op; ++i) e.pot = e.pot || ops_host[order_host[i]].v != nullptr;
  if (mix) STCHK(e.set_widths(mix->k, mix->L));
  std::vector<int> pos(chains), iters(chains, 0);
  std::vector<int64_t> fcols(chains, 0);
  std::vector<std::chrono::steady_clock::time_point> t_load(chains,
                                                            std::chrono::steady_clock::now());
  std::vector<char> active(chains, 1);
  // degree and window hint of the operator at order position `at`, loaded into slot b
  auto load_hint = [&](int b, int at) {
    int d = m;
    e.h_hint[3 * b + 2] = 0.0;
    if (hints_host) {
      const double *hh = hints_host + (size_t)order_host[at] * 3;
      const int dmax = prm->precision == SCSF_MIXED ? kMaxDegreeMixed : kMaxDegree;
      if (hh[2] >= 1.0) d = std::min(dmax, std::max(1, (int)std::lround(hh[2])));
      e.h_hint[3 * b + 0] = hh[0];
      e.h_hint[3 * b + 1] = hh[1];
      e.h_hint[3 * b + 2] = (hh[0] > 0.0 && hh[1] > 0.0) ? 1.0 : 0.0;
    }
    e.h_mraw[b] = d;
  };
  std::vector<int> all_slots(chains);
  std::iota(all_slots.begin(), all_slots.end(), 0);
  for (int b = 0; b < chains; ++b) {
    pos[b] = cb[b];
    e.h_ops[b] = to_dev(ops_host[order_host[pos[b]]]);
    e.h_need[b] = 1;
    load_hint(b, pos[b]);
  }
  STCHK(e.upload_hints(all_slots));
  STCHK(e.upload_ops());
  STCHK(e.upload_state());
  // operator index of each slot (bounds table rows)
  std::vector<int32_t> opid(chains);
  for (int b = 0; b < chains; ++b) opid[b] = order_host[pos[b]];
  if (bnd_table) STCHK(e.set_bounds(bnd_table, opid.data()));
  else STCHK(e.compute_bounds());
  {
    std::vector<int> all(chains);
    std::iota(all.begin(), all.end(), 0);
    STCHK(e.cold_start(all));
  }
  for (int b = 0; b < chains; ++b) e.h_need[b] = 0;
  STCHK(e.upload_state());

  int worst = SCSF_OK;
  int remaining = chains;
  while (remaining > 0) {
    STCHK(e.iterate());
    for (int b = 0; b < chains; ++b)
      if (active[b])
        fcols[b] += e.adaptive ? e.it_cols[b]
                               : (int64_t)(e.var_deg ? e.h_mdeg[b] : m) * (k - e.h_lock_prev(b));
    bool reload = false;
    std::vector<int> recold, reloaded;
    std::vector<std::array<int, 3>> resize;   // (slot, old side, new side)
    auto finished = [&](int b) {
      return e.h_done[b] || (e.h_flag[b] & 3) || iters[b] >= max_iter;
    };
    std::vector<int> fin_slots;
    for (int b = 0; b < chains; ++b) {
      if (!active[b]) continue;
      ++iters[b];
      if (finished(b)) fin_slots.push_back(b);
    }
    STCHK(e.fetch(fin_slots));
    // every finished problem's order and values on the host, one upload for all of them
    std::vector<double> fin_mr(chains, 0.0);
    std::vector<char> fin_cert(chains, 1);
    for (int b : fin_slots) {
      bool cert = true;
      STCHK(e.prepare_extract(b, &fin_mr[b], &cert));
      fin_cert[b] = cert ? 1 : 0;
    }
    if (!fin_slots.empty()) STCHK(e.upload_extract());
    for (int b : fin_slots) {
      const int op = order_host[pos[b]];
      const int status = solve_status(e.h_flag[b], e.h_done[b] != 0);
      double mr = 0.0;
      if (ritz) {                       // all k Ritz values, ascending
        std::vector<double> th(e.h_theta + (size_t)b * k, e.h_theta + (size_t)b * k + k);
        std::sort(th.begin(), th.end());
        HIPCHK(hipMemcpy(ritz + (size_t)op * k, th.data(), (size_t)k * 8, hipMemcpyHostToDevice));
      }
      const int64_t nop = ops_host[op].n;
      const bool cert = fin_cert[b] != 0;
      mr = fin_mr[b];
      STCHK(e.launch_extract(b, evals + (eoff ? eoff[op] : (int64_t)op * L),
                             evecs + (voff ? voff[op] : (int64_t)op * n * L), nop));
      const bool refit = low && !cert && fallback != nullptr;   // solved again, squared
      if (refit) fallback->add(op);
      if (stats_host) {
        scsf_stats &st = stats_host[op];
        st.iterations = iters[b];
        st.nconv = e.h_nconv[b] - e.off(b);
        st.status = status;
        st.chol_shifts = (e.h_flag[b] & 4) ? 1 : 0;
        st.degree = e.adaptive ? e.it_deg[b] : e.var_deg ? e.h_mdeg[b] : m;
        st.hint = (int32_t)e.h_hint[(size_t)b * 3 + 2];
        st.filter_cols = fcols[b];
        st.beta = e.h_bnd[(size_t)b * 4 + 3];
        st.max_rel_resid = mr;
        st.ms_filter = (float)e.ph[b][PH_FILTER];
        st.ms_orth = (float)e.ph[b][PH_ORTH];
        st.ms_rr = (float)e.ph[b][PH_RR];
        st.ms_resid = (float)e.ph[b][PH_RESID];
        st.ms_bound = (float)e.ph[b][PH_BOUND];
        st.ms_wall = (float)(1e3 * std::chrono::duration<double>(
                                       std::chrono::steady_clock::now() - t_load[b]).count());
        st.magnitude_route = low ? (cert ? 1 : 2) : (square ? 2 : 0);
      }
      if (!(refit && status == SCSF_ENOTCONV) && status != SCSF_OK &&
          (worst == SCSF_OK || status != SCSF_ENOTCONV))
        worst = status;
      std::atomic<int> *nx = mix ? mix->next[b] : next;   // this chain's dynamic counter
      if (nx) {
        pos[b] = nx->fetch_add(1);
      } else {
        ++pos[b];
      }
      iters[b] = 0;
      fcols[b] = 0;
      if (pos[b] >= (nx ? (mix ? mix->end[b] : n_op) : ce[b])) {
        active[b] = 0;
        --remaining;
        e.h_done[b] = 1;
        e.h_lock[b] = k;
        continue;
      }
      // next operator of the chain, warm-started from this solve (all k Ritz pairs); a
      // different size moves the vectors by bilinear interpolation (square grids) or, where
      // that is not possible, restarts cold.  cold_start, or a failed solve, restarts cold.
      const OpDev prev = e.h_ops[b];
      e.h_ops[b] = to_dev(ops_host[order_host[pos[b]]]);
      const bool bad = status == SCSF_ENUMERIC || status == SCSF_EBREAKDOWN;
      if (bad || prm->cold_start) {
        recold.push_back(b);
      } else if (e.h_ops[b].n != prev.n) {
        if (on_square_grid(prev) && on_square_grid(e.h_ops[b]))
          resize.push_back({b, prev.N, e.h_ops[b].N});
        else
          recold.push_back(b);
      }
      load_hint(b, pos[b]);
      reloaded.push_back(b);
      e.ph[b] = std::array<double, PH_COUNT>{};
      t_load[b] = std::chrono::steady_clock::now();
      e.h_need[b] = 1;
      e.h_done[b] = 0;
      e.h_nconv[b] = e.off(b);
      e.h_lock[b] = e.off(b);
      reload = true;
    }
    if (reload) {
      e.w_stale = true;                 // A X of the newly loaded operators
      STCHK(e.upload_hints(reloaded));
      STCHK(e.reset_degrees(reloaded));
      STCHK(e.upload_ops());
      for (const auto &r : resize) {
        const int64_t o = (int64_t)r[0] * e.bs;
        HIPCHK(interpolate_fields(r[1], r[2], k, e.X + o, e.ld, e.Y1 + o, e.ld, e.st));
        HIPCHK(copy_block((int64_t)r[2] * r[2], k, e.Y1 + o, e.ld, e.X + o, e.ld, false, e.st));
      }
      STCHK(e.upload_state());
      for (int b : reloaded) opid[b] = order_host[pos[b]];
      if (bnd_table) STCHK(e.set_bounds(bnd_table, opid.data()));
      else STCHK(e.compute_bounds());
      if (!recold.empty()) STCHK(e.cold_start(recold));
      for (int b = 0; b < chains; ++b) e.h_need[b] = 0;
      STCHK(e.upload_state());
    }
  }
  HIPCHK(hipStreamSynchronize(w->stream));
  return worst;
}

int add_lanes(scsf_handle *h, int count) {
  while ((int)h->ws.size() < count) {
    Workspace *w = new (std::nothrow) Workspace();
    if (!w) return SCSF_ENOMEM;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return SCSF_EHIP;
    }
    w->own_stream = true;
    w->prof = h->ws[0]->prof;
    w->arena = &h->arena;
    h->ws.push_back(w);
  }
  return SCSF_OK;
}

void free_workspace(Workspace *w) {
  (void)hipStreamSynchronize(w->stream);
  for (auto e : w->ev) (void)hipEventDestroy(e);
  for (auto &b : w->bufs)
    if (b.p && !b.in_arena) (void)hipFree(b.p);
  if (w->pinned) (void)hipHostFree(w->pinned);
  if (w->own_stream) (void)hipStreamDestroy(w->stream);
  delete w;
}

// Default block width for L wanted pairs: the smallest multiple of 8 with at least 20% guard
// vectors (Section 4 sizes the inherited subspace as a fraction of L).
static int32_t default_width(int32_t L) {
  const int32_t g = (L + 4) / 5;                       // ceil(0.2 L)
  return std::min<int32_t>(kMaxK, (int32_t)round_up(L + std::max(g, 1), 8));
}

// Autotuned settings held by the handle.
static int kbucket(int32_t k) { return k <= 48 ? 0 : k <= 96 ? 1 : k <= 160 ? 2 : 3; }
static int nbucket(int64_t n) { return n <= 4096 ? 0 : n <= 16384 ? 1 : 2; }
static int tuned_cpt(const scsf_handle *h, int64_t n, int32_t k) {
  return h->cpt[kbucket(k)][nbucket(n)];
}
static int32_t tuned_width(const scsf_handle *h, int32_t L) {
  for (const auto &p : h->widths)
    if (p.first == L) return p.second;
  return default_width(L);
}

// Scratch of scsf_bounds_noalloc (the bounds step for callers that cannot allocate): one
// operator descriptor at offset 0, the `need` flag at 256, the four bounds at 512 and the
// three Lanczos vectors (3 n doubles) from 1024.  Each GPU the library runs on holds its own
// copy until the process ends.  Host code never passes `scratch` itself (a host-side stand-in)
// to a kernel or copy: it uses the device address hipGetSymbolAddress returns for the device.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
constexpr int64_t kNoAllocMaxN = int64_t(1) << 18;
static_assert(1024 + 3 * 8 * kNoAllocMaxN <= (int64_t)kNoAllocScratchBytes, "scratch too small");
static_assert(sizeof(OpDev) <= 256, "descriptor slot too small");
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current (from scsf_create): the device address of the
// device's copy of `scratch`.
int scratch_address(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return SCSF_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return SCSF_EHIP;
    g_scratch_ptr[device] = p;
  }
  if (out) *out = g_scratch_ptr[device];
  return SCSF_OK;
}

// Device bytes the engine takes for B problems of size n (its buffers, as setup() carves them,
// each rounded up to 256 bytes).
size_t engine_bytes(int B, int64_t n, const scsf_params *p, bool var_deg) {
  Engine e;
  size_t total = 0;
  e.measure = &total;
  Workspace dummy;
  (void)e.setup(&dummy, B, n, p->k, p->L, p->degree, SCSF_STENCIL5, p->tol, p->seed, 20,
                p->precision == SCSF_MIXED, var_deg, p->adaptive != 0,
                p->target == SCSF_TARGET_MAGNITUDE);
  return total;
}

// Marks a top-level entry point: the first (outermost) one returns the caller-owned workspace's
// bump pointer to its base, since no device buffer outlives a call.
struct CallScope {
  Arena *a;
  explicit CallScope(scsf_handle *h) : a(h ? &h->arena : nullptr) {
    if (!a) return;
    std::lock_guard<std::mutex> lk(a->mu);
    if (a->depth++ == 0) {
      a->used = 0;
      ++a->gen;
    }
  }
  ~CallScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(a->mu);
    --a->depth;
  }
  CallScope(const CallScope &) = delete;
  CallScope &operator=(const CallScope &) = delete;
};

}  // namespace

// =============================================================================== C ABI
extern "C" {

const char *scsf_version(void) { return "libscsf 0.2 (gfx950, fp64 MFMA)"; }

const char *scsf_status_string(int s) {
  switch (s) {
    case SCSF_OK: return "ok";
    case SCSF_EINVAL: return "invalid argument";
    case SCSF_ENOMEM: return "out of device memory";
    case SCSF_ENOTCONV: return "not converged within max_iter";
    case SCSF_EBREAKDOWN: return "Cholesky breakdown in orthonormalisation";
    case SCSF_EHIP: return "HIP runtime error";
    case SCSF_ENUMERIC: return "NaN or Inf in the iteration";
    default: return "unknown status";
  }
}

int scsf_create(scsf_handle **h, void *hip_stream) {
  if (!h) return SCSF_EINVAL;
  scsf_handle *x = new (std::nothrow) scsf_handle();
  if (!x) return SCSF_ENOMEM;
  Workspace *w = new (std::nothrow) Workspace();
  if (!w) {
    delete x;
    return SCSF_ENOMEM;
  }
  w->stream = static_cast<hipStream_t>(hip_stream);
  w->arena = &x->arena;
  x->ws.push_back(w);
  if (hipGetDevice(&x->device) != hipSuccess) {
    delete w;
    delete x;
    return SCSF_EHIP;
  }
  (void)scratch_address(x->device, nullptr);   // scsf_bounds_noalloc reports a failure
  *h = x;
  return SCSF_OK;
}

int scsf_destroy(scsf_handle *h) {
  if (!h) return SCSF_EINVAL;
  for (auto *w : h->ws) free_workspace(w);
  delete h;
  return SCSF_OK;
}

int scsf_set_stream(scsf_handle *h, void *hip_stream) {
  if (!h) return SCSF_EINVAL;
  if (hipStreamSynchronize(h->ws[0]->stream) != hipSuccess) return SCSF_EHIP;
  h->ws[0]->stream = static_cast<hipStream_t>(hip_stream);
  return SCSF_OK;
}

int scsf_set_eigensolver(scsf_handle *h, int which) {
  if (!h || (which != SCSF_EIG_JACOBI && which != SCSF_EIG_TRIDIAG)) return SCSF_EINVAL;
  h->eig = which;
  return SCSF_OK;
}

int scsf_set_graphs(scsf_handle *h, int on) {
  if (!h) return SCSF_EINVAL;
  h->graphs = on != 0;
  return SCSF_OK;
}

int scsf_set_fused_steps(scsf_handle *h, int steps) {
  if (!h || steps < 0 || steps == 1 || steps > 4) return SCSF_EINVAL;
  h->fuse = steps;
  return SCSF_OK;
}

int scsf_set_batch_form(scsf_handle *h, int form) {
  if (!h || (form != SCSF_BATCH_GROUPED && form != SCSF_BATCH_ONE_SWEEP)) return SCSF_EINVAL;
  h->batch_form = form;
  return SCSF_OK;
}

int scsf_set_lanes(scsf_handle *h, int lanes) {
  if (!h || lanes < 1 || lanes > 16) return SCSF_EINVAL;
  h->lanes = lanes;
  return SCSF_OK;
}

int scsf_profile_enable(scsf_handle *h, int on) {
  if (!h) return SCSF_EINVAL;
  for (auto *w : h->ws) {
    if (hipStreamSynchronize(w->stream) != hipSuccess) return SCSF_EHIP;
    prof_drain(w);
    w->prof = on != 0;
  }
  return SCSF_OK;
}

int scsf_profile_read(scsf_handle *h, scsf_profile *out_host, int reset) {
  if (!h || !out_host) return SCSF_EINVAL;
  scsf_profile t{};
  for (auto *w : h->ws) {
    if (hipStreamSynchronize(w->stream) != hipSuccess) return SCSF_EHIP;
    prof_drain(w);
    t.filter_launches += w->acc.filter_launches;
    t.filter_ms += w->acc.filter_ms;
    t.filter_bytes += w->acc.filter_bytes;
    for (int p = 0; p < PH_COUNT; ++p) t.phase_ms[p] += w->phase_ms[p];
    if (reset) {
      w->acc = scsf_profile{};
      for (double &x : w->phase_ms) x = 0.0;
    }
  }
  *out_host = t;
  return SCSF_OK;
}

int scsf_workspace_bytes(const scsf_params *p, int64_t n, size_t *bytes) {
  if (!bytes || n <= 0) return SCSF_EINVAL;
  STCHK(check_params(p, n));
  *bytes = engine_bytes(1, n, p, false);
  return SCSF_OK;
}

int scsf_workspace_bytes_sequence(scsf_handle *h, const scsf_params *p, int64_t n, int32_t n_op,
                                  int32_t chains, int32_t hinted, size_t *bytes) {
  if (!h || !bytes || n <= 0 || n_op <= 0 || chains <= 0) return SCSF_EINVAL;
  STCHK(check_params(p, n));
  const int c = std::min(chains, n_op);
  const int lanes = std::min(h->lanes, c);
  size_t total = prebound_bytes(n_op, n);       // the up-front bounds (handle's own stream)
  for (int g = 0; g < lanes; ++g)
    total += engine_bytes((c - g + lanes - 1) / lanes, n, p, hinted != 0);
  *bytes = total;
  return SCSF_OK;
}

int scsf_set_workspace(scsf_handle *h, void *dev_ptr, size_t bytes) {
  if (!h || (dev_ptr && bytes == 0)) return SCSF_EINVAL;
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0) return SCSF_EINVAL;
  std::lock_guard<std::mutex> lk(h->arena.mu);
  if (h->arena.depth != 0) return SCSF_EINVAL;
  for (auto *w : h->ws) {
    if (hipStreamSynchronize(w->stream) != hipSuccess) return SCSF_EHIP;
    for (auto &b : w->bufs) {            // library-owned buffers go; carved ones are dropped
      if (b.p && !b.in_arena && hipFree(b.p) != hipSuccess) return SCSF_EHIP;
      b = DevBuf{};
    }
  }
  h->arena.base = static_cast<char *>(dev_ptr);
  h->arena.cap = dev_ptr ? bytes : 0;
  h->arena.used = 0;
  h->arena.peak = 0;
  ++h->arena.gen;
  return SCSF_OK;
}

int scsf_workspace_peak(scsf_handle *h, size_t *bytes) {
  if (!h || !bytes) return SCSF_EINVAL;
  std::lock_guard<std::mutex> lk(h->arena.mu);
  *bytes = h->arena.peak;
  return SCSF_OK;
}

int scsf_spmm(scsf_handle *h, const scsf_operator *A, const double *X, int64_t ldx, int32_t ncols,
              double *Y, int64_t ldy) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];

  STCHK(check_op(A));
  if (!X || !Y || ncols < 0 || ldx < A->n || ldy < A->n) return SCSF_EINVAL;
  if (ncols == 0) return SCSF_OK;
  Engine e;
  STCHK(e.setup(w0, 1, A->n, 1, 0, 1, A->kind, 1.0, 0, 20));
  e.h_ops[0] = to_dev(*A);
  STCHK(e.upload_ops());
  const double *src = X;
  if (ldx != ldy) {
    double *tmp = nullptr;
    STCHK(grow(w0, B_Y1, (size_t)ldy * ncols, &tmp));
    HIPCHK(copy_block(A->n, ncols, X, ldx, tmp, ldy, false, w0->stream));
    src = tmp;
  }
  HIPCHK(spmm_step(e.ops, 1, A->kind, A->n, e.Nmax, src, nullptr, Y, ldy, 0, COLS_ALL, ncols, nullptr,
                   e.unit, false, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_filter(scsf_handle *h, const scsf_operator *A, const double *X, int64_t ldx,
                int32_t ncols, int32_t degree, double lambda, double c, double e, double *Y,
                int64_t ldy) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];

  STCHK(check_op(A));
  if (!X || !Y || ncols < 0 || ncols > kMaxK || ldx < A->n || ldy < A->n) return SCSF_EINVAL;
  if (degree < 1 || degree > kMaxDegree || !(e > 0.0) || lambda == c) return SCSF_EINVAL;
  if (ncols == 0) return SCSF_OK;
  Engine en;
  STCHK(en.setup(w0, 1, A->n, ncols, 0, degree, A->kind, 1.0, 0, 20));
  en.h_ops[0] = to_dev(*A);
  STCHK(en.upload_ops());
  double *win = nullptr;
  STCHK(grow(w0, B_WIN, 3, &win));
  en.h_bnd[0] = lambda;
  en.h_bnd[1] = c;
  en.h_bnd[2] = e;
  HIPCHK(hipMemcpyAsync(win, en.h_bnd, 3 * sizeof(double), hipMemcpyHostToDevice, w0->stream));
  HIPCHK(cheb_coeffs_explicit(1, degree, win, en.coef, w0->stream));
  HIPCHK(copy_block(A->n, ncols, X, ldx, en.X, en.ld, true, w0->stream));
  double *ring[3] = {en.X, en.Y1, en.Y2};
  for (int s = 0; s < degree; ++s)
    HIPCHK(spmm_step(en.ops, 1, A->kind, A->n, en.Nmax, ring[s % 3], ring[(s + 2) % 3],
                     ring[(s + 1) % 3], en.ld, en.bs, COLS_ALL, ncols, nullptr,
                     en.coef + (size_t)s * 3, s > 0, w0->stream));
  HIPCHK(copy_block(A->n, ncols, ring[degree % 3], en.ld, Y, ldy, false, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_filter_batched(scsf_handle *h, const scsf_operator *ops_host, int32_t B,
                        const double *X, int64_t ldx, int64_t bsx, int32_t ncols, int32_t degree,
                        const double *win_host, double *Y, int64_t ldy, int64_t bsy) {
  CallScope cs_(h);
  if (!h || !ops_host || B <= 0 || !X || !Y || !win_host) return SCSF_EINVAL;
  if (ncols < 0 || ncols > kMaxK || degree < 1 || degree > kMaxDegree) return SCSF_EINVAL;
  int64_t nmax = 0;
  for (int b = 0; b < B; ++b) {
    STCHK(check_op(&ops_host[b]));
    if (ops_host[b].kind != ops_host[0].kind) return SCSF_EINVAL;
    nmax = std::max(nmax, ops_host[b].n);
    const double lam = win_host[3 * b], c = win_host[3 * b + 1], e = win_host[3 * b + 2];
    if (!(e > 0.0) || lam == c || !std::isfinite(lam) || !std::isfinite(c)) return SCSF_EINVAL;
  }
  if (ldx < nmax || ldy < nmax || bsx < ldx * (int64_t)ncols || bsy < ldy * (int64_t)ncols)
    return SCSF_EINVAL;
  if (ncols == 0) return SCSF_OK;
  // the two block ranges may not overlap
  const char *x0 = reinterpret_cast<const char *>(X), *y0 = reinterpret_cast<const char *>(Y);
  const char *x1 = x0 + ((size_t)(B - 1) * bsx + (size_t)(ncols - 1) * ldx + nmax) * 8;
  const char *y1 = y0 + ((size_t)(B - 1) * bsy + (size_t)(ncols - 1) * ldy + nmax) * 8;
  if (x0 < y1 && y0 < x1) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  Engine en;
  STCHK(en.setup(w0, B, nmax, ncols, 0, degree, ops_host[0].kind, 1.0, 0, 20));
  en.cpt = tuned_cpt(h, nmax, ncols);
  en.pot = false;
  for (int b = 0; b < B; ++b) {
    en.h_ops[b] = to_dev(ops_host[b]);
    en.pot = en.pot || ops_host[b].v != nullptr;
  }
  STCHK(en.upload_ops());
  double *win = nullptr;
  STCHK(grow(w0, B_WIN, (size_t)B * 3, &win));
  std::copy(win_host, win_host + (size_t)B * 3, en.h_bnd);     // pinned staging (B*4 doubles)
  HIPCHK(hipMemcpyAsync(win, en.h_bnd, (size_t)B * 3 * sizeof(double), hipMemcpyHostToDevice,
                        w0->stream));
  HIPCHK(cheb_coeffs_explicit(B, degree, win, en.coef, w0->stream));
  for (int b = 0; b < B; ++b)
    HIPCHK(copy_block(ops_host[b].n, ncols, X + (int64_t)b * bsx, ldx, en.X + (int64_t)b * en.bs,
                      en.ld, true, w0->stream));
  double *ring[3] = {en.X, en.Y1, en.Y2};
  en.fuse = h->fuse;
  const bool fused = en.fused_filter(degree);
  const int singles = fused ? degree % en.fuse : degree;
  for (int s = 0; s < singles; ++s) {
    const int slot = prof_begin(w0, en.step_bytes(s > 0, false, s));
    HIPCHK(spmm_step(en.ops, B, en.kind, nmax, en.Nmax, ring[s % 3], ring[(s + 2) % 3],
                     ring[(s + 1) % 3], en.ld, en.bs, COLS_ALL, ncols, nullptr,
                     en.coef + (size_t)s * B * 3, s > 0, w0->stream, nullptr, s, en.cpt, en.pot));
    prof_end(w0, slot);
  }
  if (fused) {                       // the fused schedule of the solvers (Engine::enqueue_filter)
    const Engine::FusedPlan fp = en.fused_plan(degree);
    double *cur = fp.in_cur, *prv = fp.in_prv;
    for (int g = 0, s0 = singles; s0 < degree; ++g, s0 += en.fuse) {
      double *oc = (g & 1) ? fp.odd_cur : fp.even_cur;
      double *op = (g & 1) ? fp.odd_prv : fp.even_prv;
      double bytes = 0.0;
      for (int s = s0; s < s0 + en.fuse; ++s) bytes += en.step_bytes(s > 0, false, s);
      const int slot = prof_begin(w0, bytes, en.fuse);
      HIPCHK(spmm_fused(en.ops, B, en.kind, nmax, en.Nmax, cur, s0 > 0 ? prv : nullptr, oc, op,
                        en.ld, en.bs, COLS_ALL, ncols, nullptr, en.coef + (size_t)s0 * B * 3,
                        en.fuse, w0->stream, nullptr, s0, en.cpt, en.pot));
      prof_end(w0, slot);
      cur = oc;
      prv = op;
    }
  }
  const double *res = en.filtered(degree);
  for (int b = 0; b < B; ++b)
    HIPCHK(copy_block(ops_host[b].n, ncols, res + (int64_t)b * en.bs, en.ld,
                      Y + (int64_t)b * bsy, ldy, false, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  prof_drain(w0);
  return SCSF_OK;
}

int scsf_gram_batched(scsf_handle *h, int32_t B, int64_t n, int32_t k, const double *X,
                      int64_t ldx, int64_t bsx, double *G, int32_t ldg, double *kernel_ms_host) {
  CallScope cs_(h);
  if (!h || !X || !G || B <= 0 || n <= 0 || k <= 0 || k > kMaxK || ldx < n ||
      bsx < ldx * (int64_t)k || ldg < k)
    return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  Engine en;
  STCHK(en.setup(w0, B, n, k, 0, 1, SCSF_CSR, 1.0, 0, 20));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (kernel_ms_host) {
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    HIPCHK(hipEventRecord(t0, w0->stream));
  }
  HIPCHK(gemm_tn(B, n, ldx, X, bsx, COLS_ALL, X, bsx, COLS_ALL, k, nullptr, true, en.part,
                 en.part_stride, en.G, en.ldm, nullptr, 0, w0->stream));
  if (kernel_ms_host) HIPCHK(hipEventRecord(t1, w0->stream));
  for (int b = 0; b < B; ++b)
    HIPCHK(copy_block(k, k, en.G + (int64_t)b * en.ldm * en.ldm, en.ldm,
                      G + (int64_t)b * ldg * k, ldg, false, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  if (kernel_ms_host) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    *kernel_ms_host = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
  }
  return SCSF_OK;
}

int scsf_orthonormalize(scsf_handle *h, int64_t n, double *X, int64_t ldx, int32_t ncols,
                        const double *V, int64_t ldv, int32_t nlocked) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  if (!h || n <= 0 || !X || ncols <= 0 || nlocked < 0 || ldx < n) return SCSF_EINVAL;

  if (nlocked > 0 && (!V || ldv < n)) return SCSF_EINVAL;
  const int32_t k = ncols + nlocked;
  if (k > kMaxK || k > n) return SCSF_EINVAL;
  Engine e;
  STCHK(e.setup(w0, 1, n, k, 0, 1, SCSF_STENCIL5, 1.0, 0, 20));
  if (nlocked > 0) HIPCHK(copy_block(n, nlocked, V, ldv, e.X, e.ld, true, w0->stream));
  HIPCHK(copy_block(n, ncols, X, ldx, e.X + (int64_t)nlocked * e.ld, e.ld, true, w0->stream));
  e.h_lock[0] = nlocked;
  e.h_nconv[0] = nlocked;
  STCHK(e.upload_state());
  HIPCHK(fill_int(e.flag, 0, 1, w0->stream));
  STCHK(e.orth(e.X, nlocked > 0));
  STCHK(e.download_state());
  if (e.h_flag[0] & 2) return SCSF_ENUMERIC;
  if (e.h_flag[0] & 1) return SCSF_EBREAKDOWN;
  HIPCHK(copy_block(n, ncols, e.X + (int64_t)nlocked * e.ld, e.ld, X, ldx, false, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_rayleigh_ritz(scsf_handle *h, const scsf_operator *A, double *X, int64_t ldx,
                       int32_t ncols, double *theta, double *rel_resid) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];

  STCHK(check_op(A));
  if (!X || ncols <= 0 || ncols > kMaxK || ncols > A->n || ldx < A->n) return SCSF_EINVAL;
  Engine e;
  // no locking here; the tolerance only sets the eigensolver's accuracy (full, 1e-14)
  STCHK(e.setup(w0, 1, A->n, ncols, 0, 1, A->kind, 1e-12, 0, 20));
  e.eig = h->eig;
  e.h_ops[0] = to_dev(*A);
  STCHK(e.upload_ops());
  STCHK(e.upload_state());
  HIPCHK(fill_int(e.flag, 0, 1, w0->stream));
  HIPCHK(copy_block(A->n, ncols, X, ldx, e.X, e.ld, true, w0->stream));
  STCHK(e.rayleigh_ritz(e.X));
  HIPCHK(residuals(1, A->n, e.ld, e.X, e.W, e.bs, ncols, e.lock, e.theta, e.res, w0->stream));
  HIPCHK(copy_block(A->n, ncols, e.X, e.ld, X, ldx, false, w0->stream));
  if (theta) HIPCHK(hipMemcpyAsync(theta, e.theta, (size_t)ncols * 8, hipMemcpyDeviceToDevice,
                                   w0->stream));
  if (rel_resid) HIPCHK(hipMemcpyAsync(rel_resid, e.res, (size_t)ncols * 8,
                                       hipMemcpyDeviceToDevice, w0->stream));
  STCHK(e.download_state());
  if (e.h_flag[0] & 2) return SCSF_ENUMERIC;
  return SCSF_OK;
}

int scsf_bounds(scsf_handle *h, const scsf_operator *A, int32_t steps, uint64_t seed,
                double *out_host) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  if (!h || !out_host) return SCSF_EINVAL;

  STCHK(check_op(A));
  if (steps < 1 || steps > 128) return SCSF_EINVAL;
  Engine e;
  STCHK(e.setup(w0, 1, A->n, 1, 0, 1, A->kind, 1.0, seed, steps));
  e.h_ops[0] = to_dev(*A);
  e.h_need[0] = 1;
  STCHK(e.upload_ops());
  STCHK(e.upload_state());
  HIPCHK(bounds(e.ops, 1, A->kind, A->n, steps, seed, e.need, e.lz, e.bnd, w0->stream));
  HIPCHK(hipMemcpyAsync(e.h_bnd, e.bnd, 32, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  out_host[0] = e.h_bnd[0];
  out_host[1] = e.h_bnd[1];
  out_host[2] = e.h_bnd[2];
  out_host[3] = e.h_bnd[3];
  return SCSF_OK;
}

int scsf_bounds_noalloc(scsf_handle *h, const scsf_operator *A, int32_t steps, uint64_t seed,
                        double *out_host) {
  if (!h || !out_host) return SCSF_EINVAL;
  STCHK(check_op(A));
  if (steps < 1 || steps > 128) return SCSF_EINVAL;
  if (A->n > kNoAllocMaxN) return SCSF_EINVAL;          // the Lanczos vectors would not fit
  void *base = nullptr;
  STCHK(scratch_address(h->device, &base));
  char *sb = static_cast<char *>(base);
  OpDev *op = reinterpret_cast<OpDev *>(sb);
  int32_t *need = reinterpret_cast<int32_t *>(sb + 256);
  double *bnd = reinterpret_cast<double *>(sb + 512);
  double *lz = reinterpret_cast<double *>(sb + 1024);
  hipStream_t st = h->ws[0]->stream;
  const OpDev od = to_dev(*A);
  double res[4];
  HIPCHK(hipMemcpyAsync(op, &od, sizeof(OpDev), hipMemcpyHostToDevice, st));
  HIPCHK(fill_int(need, 1, 1, st));
  HIPCHK(bounds(op, 1, A->kind, A->n, steps, seed, need, lz, bnd, st));
  HIPCHK(hipMemcpyAsync(res, bnd, sizeof(res), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < 4; ++i) out_host[i] = res[i];
  return SCSF_OK;
}

int scsf_features(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels, int32_t p,
                  int32_t p0, double *feats) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  if (!h || !fields || !feats || n_op <= 0 || channels <= 0 || p <= 0 || p0 <= 0 || p0 > p)

    return SCSF_EINVAL;
  if ((int64_t)p * p0 * 16 > 64 * 1024) return SCSF_EINVAL;
  HIPCHK(dft_features(fields, n_op, channels, p, p0, feats, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_sort(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels, int32_t p,
              int32_t p0, int32_t start, int32_t *order_host) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  if (!h || !fields || !order_host || n_op <= 0 || channels <= 0 || p <= 0 || p0 <= 0 || p0 > p)

    return SCSF_EINVAL;
  if (start < 0 || start >= n_op || n_op > 32768) return SCSF_EINVAL;
  if ((int64_t)p * p0 * 16 > 64 * 1024) return SCSF_EINVAL;
  const int32_t flen = channels * p0 * p0;
  double *F = nullptr, *D = nullptr;
  int32_t *O = nullptr;
  STCHK(grow(w0, B_SORTF, (size_t)n_op * flen * 2, &F));
  STCHK(grow(w0, B_SORTD, (size_t)n_op * n_op, &D));
  STCHK(grow(w0, B_SORTO, (size_t)n_op + 1, &O));
  HIPCHK(dft_features(fields, n_op, channels, p, p0, F, w0->stream));
  HIPCHK(pair_distances(F, n_op, flen, D, w0->stream));
  HIPCHK(greedy_order(D, n_op, start, O, w0->stream));
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(order_host, O, (size_t)n_op * 4, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipMemcpyAsync(&bad, O + n_op, 4, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return bad ? SCSF_EINVAL : SCSF_OK;
}

// One operator through Algorithm 3 on the handle's own stream (scsf_solve).  *certified is
// false for a smallest-magnitude lower-end solve whose result could not be certified.
int solve_one(scsf_handle *h, const scsf_operator *A, const scsf_params *prm,
              const double *X_prev, const double *theta_prev, double *evals, double *evecs,
              double *X_next, double *theta_next, scsf_stats *stats_host, bool square_forced,
              bool *certified, std::chrono::steady_clock::time_point t_start) {
  Workspace *w0 = h->ws[0];
  const int max_iter = prm->max_iter > 0 ? prm->max_iter : 5000;
  const int lzs = prm->lanczos_steps > 0 ? prm->lanczos_steps : 20;
  const bool low = magnitude_lower_end(prm, square_forced);
  const bool square = prm->target == SCSF_TARGET_MAGNITUDE && !low;
  Engine e;
  e.eig = h->eig;
  e.fuse = h->fuse;
  STCHK(e.setup(w0, 1, A->n, prm->k, prm->L, prm->degree, A->kind, prm->tol,
                prm->seed, lzs, prm->precision == SCSF_MIXED, false, prm->adaptive != 0,
                square));
  e.mag_low = low;
  e.h_ops[0] = to_dev(*A);
  e.h_need[0] = 1;
  STCHK(e.upload_ops());
  STCHK(e.upload_state());
  STCHK(e.compute_bounds());
  if (X_prev) {
    HIPCHK(copy_block(A->n, prm->k, X_prev, A->n, e.X, e.ld, true, w0->stream));
    HIPCHK(hipMemcpyAsync(e.theta, theta_prev, (size_t)prm->k * 8, hipMemcpyDeviceToDevice,
                          w0->stream));
  } else {
    STCHK(e.cold_start({0}));
  }
  int it = 0;
  int64_t fcols = 0;
  while (it < max_iter) {
    const int64_t uniform = (int64_t)prm->degree * (prm->k - e.h_nconv[0]);
    STCHK(e.iterate());
    fcols += e.adaptive ? e.it_cols[0] : uniform;
    ++it;
    if (e.h_done[0] || (e.h_flag[0] & 3)) break;
  }
  const bool conv = e.h_done[0] != 0;
  const int status = solve_status(e.h_flag[0], conv);
  STCHK(e.fetch(0));
  double mr = 0.0;
  bool cert = true;
  STCHK(e.extract(0, evals, evecs, A->n, &mr, &cert));
  *certified = cert;
  if (X_next) HIPCHK(copy_block(A->n, prm->k, e.X, e.ld, X_next, A->n, false, w0->stream));
  if (theta_next)
    HIPCHK(hipMemcpyAsync(theta_next, e.theta, (size_t)prm->k * 8, hipMemcpyDeviceToDevice,
                          w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  if (stats_host) {
    stats_host->iterations = it;
    stats_host->nconv = e.h_nconv[0];
    stats_host->status = status;
    stats_host->chol_shifts = (e.h_flag[0] & 4) ? 1 : 0;
    stats_host->degree = e.adaptive ? e.it_deg[0] : prm->degree;
    stats_host->hint = 0;
    stats_host->filter_cols = fcols;
    stats_host->beta = e.h_bnd[3];
    stats_host->max_rel_resid = mr;
    stats_host->ms_filter = (float)e.ph[0][PH_FILTER];
    stats_host->ms_orth = (float)e.ph[0][PH_ORTH];
    stats_host->ms_rr = (float)e.ph[0][PH_RR];
    stats_host->ms_resid = (float)e.ph[0][PH_RESID];
    stats_host->ms_bound = (float)e.ph[0][PH_BOUND];
    stats_host->ms_wall = (float)(1e3 * std::chrono::duration<double>(
                                            std::chrono::steady_clock::now() - t_start).count());
    stats_host->magnitude_route = low ? (cert ? 1 : 2) : (square ? 2 : 0);
  }
  return status;
}

int scsf_solve(scsf_handle *h, const scsf_operator *A, const scsf_params *prm,
               const double *X_prev, const double *theta_prev, double *evals, double *evecs,
               double *X_next, double *theta_next, scsf_stats *stats_host) {
  CallScope cs_(h);
  if (!h) return SCSF_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  STCHK(check_op(A));
  STCHK(check_params(prm, A->n));
  STCHK(check_op_precision(*A, prm));
  if ((X_prev == nullptr) != (theta_prev == nullptr)) return SCSF_EINVAL;
  if (!evals || !evecs) return SCSF_EINVAL;
  bool cert = true;
  const int status = solve_one(h, A, prm, X_prev, theta_prev, evals, evecs, X_next, theta_next,
                               stats_host, false, &cert, t_start);
  if (cert || (status != SCSF_OK && status != SCSF_ENOTCONV)) return status;
  // the lower end did not hold the smallest magnitudes: the squared filter, from the start
  return solve_one(h, A, prm, X_prev, theta_prev, evals, evecs, X_next, theta_next, stats_host,
                   true, &cert, t_start);
}

int scsf_solve_sequence(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                        const int32_t *order_host, int32_t chains, const scsf_params *prm,
                        double *evals, double *evecs, scsf_stats *stats_host) {
  return scsf_solve_sequence_hinted(h, ops_host, n_op, order_host, chains, prm, nullptr, evals,
                                    evecs, nullptr, stats_host);
}

int scsf_solve_sequence_hinted(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                               const int32_t *order_host, int32_t chains,
                               const scsf_params *prm, const double *hints_host, double *evals,
                               double *evecs, double *ritz, scsf_stats *stats_host) {
  CallScope cs_(h);
  if (!h || !ops_host || n_op <= 0 || !order_host || chains <= 0 || !evals || !evecs)
    return SCSF_EINVAL;
  const int64_t n = ops_host[0].n;
  const int32_t kind = ops_host[0].kind;
  for (int i = 0; i < n_op; ++i) {
    STCHK(check_op(&ops_host[i]));
    if (ops_host[i].n != n || ops_host[i].kind != kind) return SCSF_EINVAL;
  }
  STCHK(check_params(prm, n));
  STCHK(check_op_precision(ops_host[0], prm));
  if (hints_host && prm->adaptive) return SCSF_EINVAL;   // a degree hint fixes the degree
  if (hints_host && prm->target == SCSF_TARGET_MAGNITUDE) return SCSF_EINVAL;
  {
    std::vector<char> seen(n_op, 0);
    for (int i = 0; i < n_op; ++i) {
      const int o = order_host[i];
      if (o < 0 || o >= n_op || seen[o]) return SCSF_EINVAL;
      seen[o] = 1;
    }
  }
  chains = std::min(chains, n_op);
  // contiguous chunks of the order, sizes differing by at most one (App. D.6); the chunks are
  // dealt round-robin to `lanes` lockstep batches that run concurrently on their own streams
  std::vector<int> cbeg(chains + 1);
  for (int c = 0; c <= chains; ++c) cbeg[c] = (int)((int64_t)n_op * c / chains);
  const int lanes = std::min(h->lanes, chains);
  STCHK(add_lanes(h, lanes + 1));
  hipEvent_t ready;                              // the lanes start after the caller's work
  HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ready, h->ws[0]->stream));
  for (int g = 1; g <= lanes; ++g) HIPCHK(hipStreamWaitEvent(h->ws[g]->stream, ready, 0));
  std::vector<int> status(lanes, SCSF_OK);
  const bool dyn = prm->schedule == SCSF_SCHED_DYNAMIC;
  std::atomic<int> next(chains);                // dynamic: chain c starts at order position c
  Fallback fb;                                  // smallest magnitude: uncertified lower ends
  // every operator's bound in batched launches on the handle's stream, after the caller's
  // work; prebound returns once they are done, before any lane starts
  std::vector<double> btab;
  {
    const int32_t lzs = prm->lanczos_steps > 0 ? prm->lanczos_steps : 20;
    const int rc = prebound(h->ws[0], ops_host, n_op, lzs, prm->seed, btab);
    if (rc != SCSF_OK) {
      (void)hipEventDestroy(ready);
      return rc;
    }
  }
  auto lane_fn = [&](int g) {
    if (hipSetDevice(h->device) != hipSuccess) { status[g] = SCSF_EHIP; return; }
    std::vector<int> cb, ce;
    for (int c = g; c < chains; c += lanes) {
      cb.push_back(dyn ? c : cbeg[c]);
      ce.push_back(dyn ? c + 1 : cbeg[c + 1]);
    }
    status[g] = run_chains(h->ws[g + 1], ops_host, order_host, n_op, cb, ce,
                           dyn ? &next : nullptr, prm, hints_host, evals, evecs, ritz, stats_host,
                           nullptr, h->graphs, tuned_cpt(h, n, prm->k), h->eig, &fb, false,
                           h->fuse, btab.data());
  };
  std::vector<std::thread> threads;
  for (int g = 1; g < lanes; ++g) threads.emplace_back(lane_fn, g);
  lane_fn(0);
  for (auto &t : threads) t.join();
  (void)hipEventDestroy(ready);
  int worst = SCSF_OK;
  for (int g = 0; g < lanes; ++g) {
    const int s2 = status[g];
    if (s2 == SCSF_OK) continue;
    if (worst == SCSF_OK || (worst == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)) worst = s2;
  }
  if (!fb.ops.empty() && worst != SCSF_EHIP) {
    // operators whose wanted pairs were not certified at the lower end: again, with the
    // squared filter, as one chain per operator on the first lane
    std::sort(fb.ops.begin(), fb.ops.end());
    const int nf = (int)fb.ops.size();
    std::vector<int> cb(nf), ce(nf);
    std::iota(cb.begin(), cb.end(), 0);
    std::iota(ce.begin(), ce.end(), 1);
    const int s2 = run_chains(h->ws[1], ops_host, fb.ops.data(), nf, cb, ce, nullptr, prm,
                              hints_host, evals, evecs, ritz, stats_host, nullptr, h->graphs,
                              tuned_cpt(h, n, prm->k), h->eig, nullptr, true, h->fuse);
    if (s2 != SCSF_OK && (worst == SCSF_OK || (worst == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)))
      worst = s2;
  }
  return worst;
}

// ------------------------------------------------------------ uneven batches (mixed sizes)
int scsf_block_width(int32_t L) {
  if (L <= 0 || L >= kMaxK) return SCSF_EINVAL;
  return default_width(L);
}

int scsf_solve_batched(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                       const int32_t *L_host, const int32_t *k_host, const int32_t *order_host,
                       int32_t chains, const scsf_params *prm, double *evals, double *evecs,
                       scsf_stats *stats_host) {
  return scsf_solve_batched_hinted(h, ops_host, n_op, L_host, k_host, order_host, chains, prm,
                                   nullptr, evals, evecs, stats_host);
}

int scsf_solve_batched_hinted(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                              const int32_t *L_host, const int32_t *k_host,
                              const int32_t *order_host, int32_t chains,
                              const scsf_params *prm, const double *hints_host, double *evals,
                              double *evecs, scsf_stats *stats_host) {
  CallScope cs_(h);
  if (!h || !ops_host || n_op <= 0 || !L_host || !order_host || chains <= 0 || !evals ||
      !evecs || !prm)
    return SCSF_EINVAL;
  if (hints_host && (prm->adaptive || prm->target == SCSF_TARGET_MAGNITUDE)) return SCSF_EINVAL;
  const bool one_sweep = h->batch_form == SCSF_BATCH_ONE_SWEEP;
  if (one_sweep && (prm->adaptive || prm->target == SCSF_TARGET_MAGNITUDE)) return SCSF_EINVAL;
  std::vector<int32_t> kk(n_op);
  for (int i = 0; i < n_op; ++i) {
    STCHK(check_op(&ops_host[i]));
    STCHK(check_op_precision(ops_host[i], prm));
    if (L_host[i] <= 0 || L_host[i] >= kMaxK) return SCSF_EINVAL;
    kk[i] = k_host ? k_host[i] : tuned_width(h, L_host[i]);
    scsf_params p = *prm;
    p.L = L_host[i];
    p.k = kk[i];
    STCHK(check_params(&p, ops_host[i].n));
  }
  {
    std::vector<char> seen(n_op, 0);
    for (int i = 0; i < n_op; ++i) {
      const int o = order_host[i];
      if (o < 0 || o >= n_op || seen[o]) return SCSF_EINVAL;
      seen[o] = 1;
    }
  }
  // packed outputs in operator-index order
  std::vector<int64_t> eoff(n_op), voff(n_op);
  {
    int64_t e = 0, v = 0;
    for (int i = 0; i < n_op; ++i) {
      eoff[i] = e;
      voff[i] = v;
      e += L_host[i];
      v += ops_host[i].n * L_host[i];
    }
  }
  // groups of equal (kind, L, k), in order of first appearance; each keeps the given order
  struct G {
    int32_t kind, L, k;
    int64_t nmax = 0;
    std::vector<int32_t> order;
    int chains = 1;
  };
  std::vector<G> groups;
  for (int i = 0; i < n_op; ++i) {
    const int o = order_host[i];
    G *g = nullptr;
    for (auto &x : groups)
      if (x.kind == ops_host[o].kind && x.L == L_host[o] && x.k == kk[o]) g = &x;
    if (!g) {
      groups.push_back(G{ops_host[o].kind, L_host[o], kk[o]});
      g = &groups.back();
    }
    g->order.push_back(o);
    g->nmax = std::max<int64_t>(g->nmax, ops_host[o].n);
  }
  // chains shared out in proportion to the group sizes
  int maxc = 1;
  for (auto &g : groups) {
    g.chains = (int)std::lround((double)chains * (double)g.order.size() / (double)n_op);
    g.chains = std::max(1, std::min<int>(g.chains, (int)g.order.size()));
    maxc = std::max(maxc, g.chains);
  }
  const int lanes = std::min(h->lanes, maxc);
  STCHK(add_lanes(h, lanes + 1));
  hipEvent_t ready;                              // the lanes start after the caller's work
  HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ready, h->ws[0]->stream));
  for (int l = 1; l <= lanes; ++l) HIPCHK(hipStreamWaitEvent(h->ws[l]->stream, ready, 0));
  const bool dyn = prm->schedule == SCSF_SCHED_DYNAMIC;
  std::vector<std::atomic<int>> next(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) next[gi] = groups[gi].chains;
  std::vector<int> status(lanes, SCSF_OK);
  if (one_sweep) {
    // One lockstep batch per lane over the chains of every group of a kind: each sweep (outer
    // iteration) of a lane covers problems of all (L, k) of that kind at once, in the same
    // graph launches, each problem in the last k_g columns of a block as wide as the widest
    // group.  The groups' orders are concatenated; a chain keeps its group's range.
    std::vector<int32_t> kinds;
    for (const auto &g : groups)
      if (std::find(kinds.begin(), kinds.end(), g.kind) == kinds.end()) kinds.push_back(g.kind);
    struct Batch {
      std::vector<int32_t> order;
      std::vector<int> gi, head, end;            // per chain: group, first and end position
      Group grp;
    };
    std::vector<Batch> batches(kinds.size());
    for (size_t t = 0; t < kinds.size(); ++t) {
      Batch &bt = batches[t];
      bt.grp.eoff = eoff.data();
      bt.grp.voff = voff.data();
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        const G &g = groups[gi];
        if (g.kind != kinds[t]) continue;
        const int start = (int)bt.order.size(), nord = (int)g.order.size();
        bt.order.insert(bt.order.end(), g.order.begin(), g.order.end());
        for (int cc = 0; cc < g.chains; ++cc) {
          bt.gi.push_back((int)gi);
          bt.head.push_back(start + (dyn ? cc : (int)((int64_t)nord * cc / g.chains)));
          bt.end.push_back(start + (dyn ? nord : (int)((int64_t)nord * (cc + 1) / g.chains)));
        }
        next[gi] = start + g.chains;             // absolute positions in the joint order
        bt.grp.L = std::max(bt.grp.L, g.L);
        bt.grp.k = std::max(bt.grp.k, g.k);
        bt.grp.nmax = std::max(bt.grp.nmax, g.nmax);
      }
    }
    auto sweep_fn = [&](int l) {
      if (hipSetDevice(h->device) != hipSuccess) { status[l] = SCSF_EHIP; return; }
      const size_t nb = batches.size();
      for (size_t j = 0; j < nb; ++j) {
        const Batch &bt = batches[(j + (size_t)l) % nb];
        std::vector<int> cb, ce;
        Mix mix;
        for (size_t cc = (size_t)l; cc < bt.gi.size(); cc += (size_t)lanes) {
          const G &g = groups[bt.gi[cc]];
          cb.push_back(bt.head[cc]);
          ce.push_back(dyn ? bt.head[cc] + 1 : bt.end[cc]);
          mix.L.push_back(g.L);
          mix.k.push_back(g.k);
          mix.next.push_back(dyn ? &next[bt.gi[cc]] : nullptr);
          mix.end.push_back(bt.end[cc]);
        }
        if (cb.empty()) continue;
        const int s2 = run_chains(h->ws[l + 1], ops_host, bt.order.data(), (int)bt.order.size(),
                                  cb, ce, nullptr, prm, hints_host, evals, evecs, nullptr,
                                  stats_host, &bt.grp, h->graphs,
                                  tuned_cpt(h, bt.grp.nmax, bt.grp.k), h->eig, nullptr, false,
                                  h->fuse, nullptr, &mix);
        if (s2 != SCSF_OK && (status[l] == SCSF_OK ||
                              (status[l] == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)))
          status[l] = s2;
        if (s2 != SCSF_OK && s2 != SCSF_ENOTCONV) return;
      }
    };
    std::vector<std::thread> threads;
    for (int l = 1; l < lanes; ++l) threads.emplace_back(sweep_fn, l);
    sweep_fn(0);
    for (auto &t : threads) t.join();
    (void)hipEventDestroy(ready);
    int worst = SCSF_OK;
    for (int l = 0; l < lanes; ++l) {
      const int s2 = status[l];
      if (s2 == SCSF_OK) continue;
      if (worst == SCSF_OK || (worst == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)) worst = s2;
    }
    return worst;
  }
  std::vector<Fallback> fbs(groups.size());     // smallest magnitude: uncertified lower ends
  // every lane works through the groups in turn, starting at group l mod G, so all groups are
  // in flight from the start (narrow groups' dense steps overlap wide groups' filters); a lane
  // that finishes its chains of one group moves on to the next without waiting for the others
  const size_t ng = groups.size();
  auto lane_fn = [&](int l) {
    if (hipSetDevice(h->device) != hipSuccess) { status[l] = SCSF_EHIP; return; }
    for (size_t j = 0; j < ng; ++j) {
      const size_t gi = (j + (size_t)l) % ng;
      const G &g = groups[gi];
      const int nord = (int)g.order.size();
      std::vector<int> cb, ce;
      for (int c = l; c < g.chains; c += lanes) {
        cb.push_back(dyn ? c : (int)((int64_t)nord * c / g.chains));
        ce.push_back(dyn ? c + 1 : (int)((int64_t)nord * (c + 1) / g.chains));
      }
      if (cb.empty()) continue;
      Group grp;
      grp.L = g.L;
      grp.k = g.k;
      grp.nmax = g.nmax;
      grp.eoff = eoff.data();
      grp.voff = voff.data();
      const int s2 = run_chains(h->ws[l + 1], ops_host, g.order.data(), nord, cb, ce,
                                dyn ? &next[gi] : nullptr, prm, hints_host, evals, evecs, nullptr,
                                stats_host, &grp, h->graphs, tuned_cpt(h, g.nmax, g.k), h->eig,
                                &fbs[gi], false, h->fuse);
      if (s2 != SCSF_OK && (status[l] == SCSF_OK ||
                            (status[l] == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)))
        status[l] = s2;
      if (s2 != SCSF_OK && s2 != SCSF_ENOTCONV) return;
    }
  };
  std::vector<std::thread> threads;
  for (int l = 1; l < lanes; ++l) threads.emplace_back(lane_fn, l);
  lane_fn(0);
  for (auto &t : threads) t.join();
  (void)hipEventDestroy(ready);
  int worst = SCSF_OK;
  for (int l = 0; l < lanes; ++l) {
    const int s2 = status[l];
    if (s2 == SCSF_OK) continue;
    if (worst == SCSF_OK || (worst == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)) worst = s2;
  }
  // uncertified smallest-magnitude solves again with the squared filter, one chain each
  for (size_t gi = 0; gi < groups.size() && worst != SCSF_EHIP; ++gi) {
    auto &fo = fbs[gi].ops;
    if (fo.empty()) continue;
    std::sort(fo.begin(), fo.end());
    const int nf = (int)fo.size();
    std::vector<int> cb(nf), ce(nf);
    std::iota(cb.begin(), cb.end(), 0);
    std::iota(ce.begin(), ce.end(), 1);
    Group grp;
    grp.L = groups[gi].L;
    grp.k = groups[gi].k;
    grp.nmax = groups[gi].nmax;
    grp.eoff = eoff.data();
    grp.voff = voff.data();
    const int s2 = run_chains(h->ws[1], ops_host, fo.data(), nf, cb, ce, nullptr, prm, nullptr,
                              evals, evecs, nullptr, stats_host, &grp, h->graphs,
                              tuned_cpt(h, grp.nmax, grp.k), h->eig, nullptr, true, h->fuse);
    if (s2 != SCSF_OK && (worst == SCSF_OK || (worst == SCSF_ENOTCONV && s2 != SCSF_ENOTCONV)))
      worst = s2;
  }
  return worst;
}

// ---- autotuner
// SpMM tile: time the filter step on B copies of a representative operator for each
// columns-per-thread choice and keep the fastest.
static int tune_tile(Workspace *w, const scsf_operator &rep, int32_t k, int32_t *best) {
  constexpr int reps = 10;
  // enough copies for a working set of about 768 MB (the 256 MB MALL must not hold it)
  const double blk = 3.0 * 8.0 * (double)round_up(rep.n, 64) * k;
  const int B = (int)std::min<double>(64.0, std::max(8.0, std::ceil(768e6 / blk)));
  Engine e;
  STCHK(e.setup(w, B, rep.n, k, 1, 1, rep.kind, 1.0, 7, 20));
  for (int b = 0; b < B; ++b) e.h_ops[b] = to_dev(rep);
  STCHK(e.upload_ops());
  HIPCHK(gaussian_fill(B, rep.n, e.ld, e.bs, k, e.X, 0x7A11ULL, e.st));
  HIPCHK(gaussian_fill(B, rep.n, e.ld, e.bs, k, e.Y2, 0x7A12ULL, e.st));
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return SCSF_EHIP;
  }
  float best_ms = 1e30f;
  int rc = SCSF_OK;
  *best = 4;
  for (int c : {4, 2, 1}) {            // the default first: another tile must beat it by 10%
    auto step = [&] {
      return spmm_step(e.ops, B, e.kind, e.n, e.Nmax, e.X, e.Y2, e.Y1, e.ld, e.bs, COLS_ALL, k,
                       nullptr, e.unit, true, e.st, nullptr, 0, c, rep.v != nullptr);
    };
    if (step() != hipSuccess) { rc = SCSF_EHIP; break; }
    if (hipEventRecord(t0, e.st) != hipSuccess) { rc = SCSF_EHIP; break; }
    for (int r = 0; r < reps; ++r)
      if (step() != hipSuccess) rc = SCSF_EHIP;
    if (rc != SCSF_OK || hipEventRecord(t1, e.st) != hipSuccess ||
        hipEventSynchronize(t1) != hipSuccess) { rc = SCSF_EHIP; break; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t0, t1) != hipSuccess) { rc = SCSF_EHIP; break; }
    if (c == 4) best_ms = ms;
    else if (ms < 0.90f * best_ms) { best_ms = ms; *best = c; }
  }
  (void)hipStreamSynchronize(e.st);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return rc;
}

// Block width for L: a warm-started probe chain over the group's first operators for each
// candidate width; the width with the least time per eigenpair wins.
static int tune_width(scsf_handle *h, Workspace *w, const scsf_operator *ops_host, int32_t n_op,
                      const std::vector<int32_t> &probe, int32_t L, const scsf_params *prm,
                      int32_t *best) {
  int64_t nmin = INT64_MAX, nmax = 0, ne = 0, nv = 0;
  std::vector<int64_t> eoff(n_op, 0), voff(n_op, 0);
  for (int o : probe) {
    nmin = std::min<int64_t>(nmin, ops_host[o].n);
    nmax = std::max<int64_t>(nmax, ops_host[o].n);
    eoff[o] = ne;
    voff[o] = nv;
    ne += L;
    nv += ops_host[o].n * L;
  }
  std::vector<int32_t> cand;
  for (double f : {1.2, 1.35, 1.5}) {
    const int32_t kc = (int32_t)round_up((int64_t)std::ceil(f * L), 8);
    if (kc > L && kc <= kMaxK && kc <= nmin &&
        std::find(cand.begin(), cand.end(), kc) == cand.end())
      cand.push_back(kc);
  }
  *best = default_width(L);
  if (cand.empty()) return SCSF_OK;
  double *ev = nullptr, *vv = nullptr;           // probe outputs (buffers the engine leaves alone)
  STCHK(grow(w, B_TEV, (size_t)ne, &ev));
  STCHK(grow(w, B_TVV, (size_t)nv, &vv));
  double best_t = 1e300;
  int rc = SCSF_OK;
  for (int32_t kc : cand) {
    scsf_params p = *prm;
    p.L = L;
    p.k = kc;
    Group grp;
    grp.L = L;
    grp.k = kc;
    grp.nmax = nmax;
    grp.eoff = eoff.data();
    grp.voff = voff.data();
    std::vector<int> cb{0}, ce{(int)probe.size()};
    const auto t0 = std::chrono::steady_clock::now();
    const int s2 = run_chains(w, ops_host, probe.data(), (int32_t)probe.size(), cb, ce, nullptr,
                              &p, nullptr, ev, vv, nullptr, nullptr, &grp, h->graphs,
                              tuned_cpt(h, nmax, kc), h->eig, nullptr, false, h->fuse);
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (s2 == SCSF_ENOTCONV) continue;             // a width that cannot converge never wins
    if (s2 != SCSF_OK) { rc = s2; break; }
    if (dt < best_t) { best_t = dt; *best = kc; }
  }
  return rc;
}

int scsf_autotune(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                  const int32_t *L_host, const int32_t *order_host, const scsf_params *prm,
                  int32_t probe) {
  CallScope cs_(h);
  if (!h || !ops_host || n_op <= 0 || !L_host || !order_host || !prm || probe < 1 || probe > 64)
    return SCSF_EINVAL;
  if (prm->precision != SCSF_FP64) return SCSF_EINVAL;
  for (int i = 0; i < n_op; ++i) {
    STCHK(check_op(&ops_host[i]));
    if (L_host[i] <= 0 || L_host[i] >= kMaxK) return SCSF_EINVAL;
    scsf_params p = *prm;
    p.L = L_host[i];
    p.k = std::min<int64_t>(default_width(L_host[i]), ops_host[i].n);
    if (p.k <= p.L) return SCSF_EINVAL;
    STCHK(check_params(&p, ops_host[i].n));
  }
  {
    std::vector<char> seen(n_op, 0);
    for (int i = 0; i < n_op; ++i) {
      const int o = order_host[i];
      if (o < 0 || o >= n_op || seen[o]) return SCSF_EINVAL;
      seen[o] = 1;
    }
  }
  STCHK(add_lanes(h, 2));
  Workspace *w = h->ws[1];
  HIPCHK(hipStreamSynchronize(h->ws[0]->stream));
  bool tuned[4][3] = {};
  std::vector<int32_t> Ls;
  for (int i = 0; i < n_op; ++i) {
    const int32_t L = L_host[order_host[i]];
    if (std::find(Ls.begin(), Ls.end(), L) == Ls.end()) Ls.push_back(L);
  }
  for (int32_t L : Ls) {
    // operators with this L and the kind of the first of them, in the given order
    std::vector<int32_t> grp;
    int32_t kind = 0;
    for (int i = 0; i < n_op; ++i) {
      const int o = order_host[i];
      if (L_host[o] != L) continue;
      if (grp.empty()) kind = ops_host[o].kind;
      if (ops_host[o].kind == kind) grp.push_back(o);
    }
    // tiles for every (width candidate, size bucket) this group meets
    for (double f : {1.2, 1.35, 1.5}) {
      const int32_t kc = (int32_t)round_up((int64_t)std::ceil(f * L), 8);
      if (kc > kMaxK) continue;
      for (int nb = 0; nb < 3; ++nb) {
        if (tuned[kbucket(kc)][nb]) continue;
        int rep = -1;
        for (int o : grp)
          if (nbucket(ops_host[o].n) == nb && ops_host[o].n >= kc &&
              (rep < 0 || ops_host[o].n > ops_host[rep].n))
            rep = o;
        if (rep < 0) continue;
        int32_t c = 4;
        STCHK(tune_tile(w, ops_host[rep], kc, &c));
        h->cpt[kbucket(kc)][nb] = c;
        tuned[kbucket(kc)][nb] = true;
      }
    }
    std::vector<int32_t> pr(grp.begin(), grp.begin() + std::min<size_t>(grp.size(), probe));
    int32_t kbest = default_width(L);
    STCHK(tune_width(h, w, ops_host, n_op, pr, L, prm, &kbest));
    bool found = false;
    for (auto &p : h->widths)
      if (p.first == L) { p.second = kbest; found = true; }
    if (!found) h->widths.emplace_back(L, kbest);
  }
  return SCSF_OK;
}

int scsf_set_tile(scsf_handle *h, int32_t tile) {
  if (!h || (tile != 1 && tile != 2 && tile != 4 && tile != 8)) return SCSF_EINVAL;
  for (auto &row : h->cpt)
    for (auto &c : row) c = tile;
  return SCSF_OK;
}

int scsf_tuned_width(scsf_handle *h, int32_t L) {
  if (!h || L <= 0 || L >= kMaxK) return SCSF_EINVAL;
  return tuned_width(h, L);
}

int scsf_tuned_tile(scsf_handle *h, int64_t n, int32_t k) {
  if (!h || n <= 0 || k <= 0 || k > kMaxK) return SCSF_EINVAL;
  return tuned_cpt(h, n, k);
}

int scsf_interpolate(scsf_handle *h, int32_t N0, int32_t N1, int32_t ncols, const double *X,
                     int64_t ldx, double *Y, int64_t ldy) {
  CallScope cs_(h);
  if (!h || N0 <= 0 || N1 <= 0 || ncols < 0 || ncols > 65535) return SCSF_EINVAL;
  if (ncols == 0) return SCSF_OK;
  if (!X || !Y || ldx < (int64_t)N0 * N0 || ldy < (int64_t)N1 * N1) return SCSF_EINVAL;
  // no overlap between the source and destination ranges
  const char *x0 = reinterpret_cast<const char *>(X);
  const char *x1 = reinterpret_cast<const char *>(X + (int64_t)(ncols - 1) * ldx + (int64_t)N0 * N0);
  const char *y0 = reinterpret_cast<const char *>(Y);
  const char *y1 = reinterpret_cast<const char *>(Y + (int64_t)(ncols - 1) * ldy + (int64_t)N1 * N1);
  if (x0 < y1 && y0 < x1) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(interpolate_fields(N0, N1, ncols, X, ldx, Y, ldy, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_highfreq_ratio(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels,
                        int32_t p, int32_t p0, double *ratio) {
  CallScope cs_(h);
  if (!h || !fields || !ratio || n_op <= 0 || channels <= 0 || p <= 0 || p0 <= 0)
    return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(highfreq_ratio(fields, n_op, channels, p, p0, ratio, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_subspace_distance(scsf_handle *h, int64_t n, int32_t q, const double *X, int64_t ldx,
                           int64_t bsx, int32_t n_blocks, const int32_t *a_host,
                           const int32_t *b_host, int32_t P, double *out_host) {
  CallScope cs_(h);
  if (!h || !X || !a_host || !b_host || !out_host || n <= 0 || q <= 0 || q > kMaxDistQ ||
      q > n || ldx < n || bsx < ldx * (int64_t)q || n_blocks <= 0 || P < 0)
    return SCSF_EINVAL;
  for (int i = 0; i < P; ++i)
    if (a_host[i] < 0 || a_host[i] >= n_blocks || b_host[i] < 0 || b_host[i] >= n_blocks)
      return SCSF_EINVAL;
  if (P == 0) return SCSF_OK;
  Workspace *w0 = h->ws[0];
  int32_t *idx = nullptr;
  double *out = nullptr;
  STCHK(grow(w0, B_SORTO, (size_t)2 * P, &idx));
  STCHK(grow(w0, B_SORTD, (size_t)P, &out));
  HIPCHK(hipMemcpyAsync(idx, a_host, (size_t)P * 4, hipMemcpyHostToDevice, w0->stream));
  HIPCHK(hipMemcpyAsync(idx + P, b_host, (size_t)P * 4, hipMemcpyHostToDevice, w0->stream));
  HIPCHK(subspace_distance(n, q, X, ldx, bsx, idx, idx + P, P, out, w0->stream));
  HIPCHK(hipMemcpyAsync(out_host, out, (size_t)P * 8, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_order_features(scsf_handle *h, const double *feats, int32_t n_op, int32_t flen,
                        int32_t start, int32_t *order_host) {
  CallScope cs_(h);
  if (!h || !feats || !order_host || n_op <= 0 || flen <= 0) return SCSF_EINVAL;
  if (start < 0 || start >= n_op || n_op > 32768) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  double *D = nullptr;
  int32_t *O = nullptr;
  STCHK(grow(w0, B_SORTD, (size_t)n_op * n_op, &D));
  STCHK(grow(w0, B_SORTO, (size_t)n_op + 1, &O));
  HIPCHK(pair_distances(feats, n_op, flen, D, w0->stream));
  HIPCHK(greedy_order(D, n_op, start, O, w0->stream));
  int32_t bad = 0;
  HIPCHK(hipMemcpyAsync(order_host, O, (size_t)n_op * 4, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipMemcpyAsync(&bad, O + n_op, 4, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return bad ? SCSF_EINVAL : SCSF_OK;
}

// ------------------------------------------------------------------ the learned window
int scsf_window_param_count(void) { return (int)kNetParams; }

namespace {
struct NetBufs {
  float *a1, *a2, *a3, *y, *d, *da3, *da2, *da1, *grad, *m, *v;
  uint16_t *pbf, *xbf, *b1, *b2, *b3, *ybf;
  double *loss;
};
int net_bufs(Workspace *w, int n, NetBufs &nb) {
  const size_t per = 4096 + 2048 + 64 + 3 + 3 + 64 + 2048 + 4096;
  float *f = nullptr;
  STCHK(grow(w, B_NETF, (size_t)n * per + 3 * (size_t)kNetParams + 64, &f));
  nb.a1 = f; f += (size_t)n * 4096;
  nb.a2 = f; f += (size_t)n * 2048;
  nb.a3 = f; f += (size_t)n * 64;
  nb.y = f; f += (size_t)n * 3;
  nb.d = f; f += (size_t)n * 3;
  nb.da3 = f; f += (size_t)n * 64;
  nb.da2 = f; f += (size_t)n * 2048;
  nb.da1 = f; f += (size_t)n * 4096;
  nb.grad = f; f += kNetParams;
  nb.m = f; f += kNetParams;
  nb.v = f;
  uint16_t *hh = nullptr;
  STCHK(grow(w, B_NETH, (size_t)kNetParams + (size_t)n * (1536 + 4096 + 2048 + 64 + 3) + 64, &hh));
  nb.pbf = hh; hh += kNetParams;
  nb.xbf = hh; hh += (size_t)n * 1536;
  nb.b1 = hh; hh += (size_t)n * 4096;
  nb.b2 = hh; hh += (size_t)n * 2048;
  nb.b3 = hh; hh += (size_t)n * 64;
  nb.ybf = hh;
  STCHK(grow(w, B_NETD, 8, &nb.loss));
  return SCSF_OK;
}
}  // namespace

int scsf_window_init(scsf_handle *h, float *params, uint64_t seed) {
  CallScope cs_(h);
  if (!h || !params) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(cnn_init(params, seed, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_input(scsf_handle *h, const double *feats, int32_t n, int32_t channels,
                      int32_t p0, float *x) {
  CallScope cs_(h);
  if (!h || !feats || !x || n <= 0 || channels != 3 || p0 != 16) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(cnn_input(feats, n, channels, p0, x, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_forward(scsf_handle *h, const float *params, const float *x, int32_t n,
                        int32_t bf16, float *out) {
  CallScope cs_(h);
  if (!h || !params || !x || !out || n <= 0) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  NetBufs nb;
  STCHK(net_bufs(w0, n, nb));
  if (bf16)
    HIPCHK(cnn_forward_bf16(params, x, n, nb.pbf, nb.xbf, nb.b1, nb.b2, nb.b3, nb.ybf, out,
                            w0->stream));
  else
    HIPCHK(cnn_forward(params, x, n, nb.a1, nb.a2, nb.a3, out, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_loss_grad(scsf_handle *h, const float *params, const float *x,
                          const float *target, int32_t n, float *grad, double *loss_host) {
  CallScope cs_(h);
  if (!h || !params || !x || !target || !grad || n <= 0) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  NetBufs nb;
  STCHK(net_bufs(w0, n, nb));
  HIPCHK(cnn_loss_grad(params, x, target, n, nb.a1, nb.a2, nb.a3, nb.y, nb.d, nb.da3, nb.da2,
                       nb.da1, grad, nb.loss, w0->stream));
  if (loss_host)
    HIPCHK(hipMemcpyAsync(loss_host, nb.loss, 8, hipMemcpyDeviceToHost, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_train(scsf_handle *h, float *params, const float *x, const float *target,
                      int32_t n, int32_t epochs, float lr, double *loss_history_host) {
  CallScope cs_(h);
  if (!h || !params || !x || !target || n <= 0 || epochs <= 0 || !(lr > 0.f)) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  NetBufs nb;
  STCHK(net_bufs(w0, n, nb));
  // the epochs' losses stay on the device until the end (no per-epoch synchronisation)
  double *hist = nullptr;
  STCHK(grow(w0, B_NETL, (size_t)epochs, &hist));
  HIPCHK(hipMemsetAsync(nb.m, 0, (size_t)2 * kNetParams * sizeof(float), w0->stream));
  for (int ep = 1; ep <= epochs; ++ep) {
    HIPCHK(cnn_loss_grad(params, x, target, n, nb.a1, nb.a2, nb.a3, nb.y, nb.d, nb.da3, nb.da2,
                         nb.da1, nb.grad, hist + (ep - 1), w0->stream));
    HIPCHK(cnn_adam(params, nb.grad, nb.m, nb.v, ep, lr, w0->stream));
  }
  if (loss_history_host)
    HIPCHK(hipMemcpyAsync(loss_history_host, hist, (size_t)epochs * 8, hipMemcpyDeviceToHost,
                          w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_labels(scsf_handle *h, const double *ritz, int32_t n, int32_t k, int32_t L,
                       const double *beta, float *target) {
  CallScope cs_(h);
  if (!h || !ritz || !beta || !target || n <= 0 || L <= 0 || L >= k) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(cnn_labels(ritz, n, k, L, beta, target, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

int scsf_window_hints(scsf_handle *h, const float *out, int32_t n, double *hints) {
  CallScope cs_(h);
  if (!h || !out || !hints || n <= 0) return SCSF_EINVAL;
  Workspace *w0 = h->ws[0];
  HIPCHK(cnn_hints(out, n, hints, w0->stream));
  HIPCHK(hipStreamSynchronize(w0->stream));
  return SCSF_OK;
}

}  // extern "C"
