/*
 * scsf.h -- C ABI of the MI355X (gfx950) SCSF hot-path library, libscsf.so.
 *
 * SCSF (arXiv 2510.23215) generates eigenvalue datasets: it orders a sequence of sparse
 * symmetric operators A^(i) by a truncated-FFT greedy sort (Algorithm 2) and solves each for
 * its L smallest eigenpairs (eq. eq_basic, Section 2.1) with Chebyshev filtered subspace
 * iteration (Algorithm 3), warm-started from the previous operator's eigenpairs.
 *
 * Conventions for every entry point
 *   - Pointers whose name ends in `_host` are host memory; every other array argument is
 *     DEVICE memory on the handle's device.  The caller owns every buffer it passes; the
 *     handle owns only its internal workspace (device memory it allocates and reuses, or a
 *     caller-owned area given with scsf_set_workspace).
 *   - Blocks of vectors are column-major with leading dimension `ld` >= n (element (i, j) at
 *     X[i + j*ld]).  Small matrices are column-major, leading dimension = their row count.
 *   - Work is enqueued on the handle's stream.  Entry points that must read a device-side
 *     result (lock counts, the sort order, bounds) synchronise that stream before returning.
 *   - Every entry point returns an scsf status (0 = success, negative = error).  On an error
 *     other than SCSF_ENOTCONV the outputs are unspecified and the handle stays usable.
 *   - Nothing here is thread-safe per handle; use one handle per host thread.
 */
#ifndef SCSF_H
#define SCSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct scsf_handle scsf_handle;

enum scsf_status {
  SCSF_OK = 0,
  SCSF_EINVAL = -1,      /* an argument is out of range (sizes, NULL where not allowed) */
  SCSF_ENOMEM = -2,      /* device workspace could not be allocated */
  SCSF_ENOTCONV = -3,    /* max_iter reached; best pairs so far were written */
  SCSF_EBREAKDOWN = -4,  /* Cholesky of a Gram matrix failed even with a shift */
  SCSF_EHIP = -5,        /* a HIP runtime call failed */
  SCSF_ENUMERIC = -6     /* NaN or Inf met in the iteration */
};

enum scsf_op_kind {
  SCSF_STENCIL5 = 1,     /* conservative 5-point -div(K grad u) + v u on an nx x nx grid */
  SCSF_STENCIL9 = 2,     /* 9-point Q1 stiffness of cell tensors / h^2 on an nx x nx grid */
  SCSF_CSR = 3,          /* general symmetric CSR matrix (both triangles stored) */
  SCSF_PLATE = 4         /* thin-plate vibration del^2(D del^2 u) = lambda rho u (App. D.2) in
                            standard form M^{-1/2} K M^{-1/2} on an nx x nx grid */
};

enum scsf_precision { SCSF_FP64 = 0, SCSF_MIXED = 1 };

/* How scsf_solve_sequence hands operators to its concurrent chains.
 *   STATIC : the sorted order is cut into `chains` contiguous chunks (App. D.6 chunking);
 *   DYNAMIC: every chain takes the next unsolved operator of the sorted order when it
 *            finishes one, warm-starting from the operator it solved last (load balance). */
enum scsf_schedule { SCSF_SCHED_STATIC = 0, SCSF_SCHED_DYNAMIC = 1 };
/* How scsf_solve_batched runs operators with different (L, k) (scsf_set_batch_form). */
enum scsf_batch_form { SCSF_BATCH_GROUPED = 0, SCSF_BATCH_ONE_SWEEP = 1 };
/* Which eigenvalues the solvers return (scsf_params.target). */
enum scsf_target { SCSF_TARGET_SMALLEST = 0, SCSF_TARGET_MAGNITUDE = 1 };
/* Eigensolver of the Rayleigh-Ritz step (scsf_set_eigensolver). */
enum scsf_eigensolver { SCSF_EIG_JACOBI = 0, SCSF_EIG_TRIDIAG = 1 };

/*
 * A discretised operator (Section 2.1; datasets of App. D.2).  Grid nodes are numbered
 * row-major, p = iy*nx + ix, h = 1/(nx+1), zero Dirichlet values beyond the boundary.
 *   STENCIL5: wx[iy*(nx+1) + f] is the coefficient of the x-face between nodes (iy, f-1) and
 *             (iy, f) (f = 0 and f = nx are boundary faces); wy[f*nx + ix] the y-face between
 *             (f-1, ix) and (f, ix); v[p] an optional diagonal term (NULL = 0).  The matrix is
 *             (A u)_p = sum_faces w (u_p - u_nbr) + v_p u_p; coefficients carry 1/h^2.
 *   STENCIL9: cell[(cy*(nx+1) + cx)*3 + {0,1,2}] = (K11, K12, K22) of cell (cy, cx), the square
 *             between node rows cy-1, cy and columns cx-1, cx; A = Q1 stiffness / h^2.
 *   CSR:      row_ptr[n+1], col_idx[nnz], val[nnz], symmetric.
 *   PLATE:    wx[p] = flexural rigidity D > 0 and wy[p] = density rho > 0 at node p (n each);
 *             v must be NULL.  K = L diag(D) L with L the 5-point Dirichlet Laplacian / h^2
 *             (simply supported edges: u = 0 and del^2 u = 0 on the boundary), M = diag(rho)
 *             (lumped mass).  The solvers work on A = M^{-1/2} K M^{-1/2} (same eigenvalues,
 *             A y = lambda y with y = M^{1/2} u) and return u = M^{-1/2} y, M-orthonormal
 *             (u^T M u = I); warm-start blocks (X_prev / X_next) and scsf_spmm / scsf_filter
 *             use the standard-form vectors y, and residuals are those of A.  FP64 only
 *             (SCSF_MIXED gives SCSF_EINVAL); nx <= 600.
 * All coefficient arrays are device memory and must stay valid during the call.
 */
typedef struct scsf_operator {
  int32_t kind;
  int32_t nx;            /* grid side for the stencil kinds (n = nx*nx); 0 for CSR */
  int64_t n;             /* matrix dimension */
  const double *wx, *wy, *v;
  const double *cell;
  const int32_t *row_ptr, *col_idx;
  const double *val;
  int64_t nnz;
} scsf_operator;

/* Solver parameters (Algorithm 3; defaults of App. D.4: degree 20, k = L + 20% of L). */
typedef struct scsf_params {
  int32_t L;             /* wanted eigenpairs, 0 < L < k */
  int32_t k;             /* block width (L + guard vectors), k <= n, k <= 256 */
  int32_t degree;        /* Chebyshev degree m, 1..128 (1..64 with SCSF_MIXED) */
  int32_t max_iter;      /* outer iterations before SCSF_ENOTCONV (0 -> 5000) */
  int32_t lanczos_steps; /* steps of the upper-bound Lanczos run (0 -> 20) */
  int32_t precision;     /* scsf_precision */
  int32_t schedule;      /* scsf_solve_sequence: scsf_schedule */
  int32_t adaptive;      /* 1: per-vector filter degrees (the optimized filter cited for
                            Algorithm 1): after an outer iteration every active column gets
                            ceil(ln(res/tol) / ln|rho|) steps, |rho| = |t| + sqrt(t^2 - 1),
                            t = (theta - c) / e, clamped to [degree, min(2 degree, 64)] and
                            raised by at most 2 to the residue mod 3 of the iteration's largest
                            degree.  FP64 only; not with degree hints (SCSF_EINVAL).  0: one
                            degree for the whole block */
  int32_t cold_start;    /* chained solvers: 0 -> each solve of a chain starts from the previous
                            solve's k Ritz pairs (Section 3.2); 1 -> every solve starts from a
                            seeded random block (the unsorted, cold baseline of the paper's
                            ablations) */
  int32_t target;        /* scsf_target: SCSF_TARGET_SMALLEST, the L algebraically smallest
                            eigenvalues; SCSF_TARGET_MAGNITUDE, the L smallest in absolute
                            value (indefinite operators, the Helmholtz family of App. D.2),
                            evals ordered by |lambda| (signed).  Two routes: (1) when L + 1 < k,
                            the plain method for the L + 1 algebraically smallest pairs; their L
                            of smallest |lambda| are returned when |lambda_1| <= lambda_{L+1},
                            which proves them the L smallest in magnitude (a short negative
                            spectrum, as in the Helmholtz datasets); (2) otherwise, or when that
                            certificate fails (the operator is then solved again from the
                            start), the filter runs on A^2 (each Chebyshev step applies A
                            twice, window and bound squared) while Rayleigh-Ritz, residuals and
                            locking stay with A (slow on wide spectra: it squares their
                            spread).  scsf_stats.magnitude_route says which.  FP64 only; not
                            with adaptive degrees or degree hints */
  double tol;            /* lock when ||A v - theta v|| <= tol ||A v|| (App. D.5 metric) */
  uint64_t seed;         /* seed of the random cold-start block and Lanczos start vector */
} scsf_params;

/* Per-solve statistics (host struct). */
typedef struct scsf_stats {
  int32_t iterations;    /* outer iterations */
  int32_t nconv;         /* locked pairs at exit (>= L on success) */
  int32_t status;        /* status of this solve */
  int32_t chol_shifts;   /* Gram matrices that needed the shifted Cholesky fallback */
  int32_t degree;        /* filter degree used (last iteration) */
  int32_t hint;          /* window hint: 0 none, 2 used, 3 rejected by the Lanczos bounds */
  int64_t filter_cols;   /* sum over filter calls of degree * active columns */
  double beta;           /* upper spectral bound used by the filter */
  double max_rel_resid;  /* max relative residual of the returned pairs */
  /* Device time of each step of Algorithm 3 for this solve (HIP events on the stream the
   * solve ran on; the cost split of App. E.3).  In the chained and batched solvers the
   * launches are shared by the problems of a lockstep batch, and each problem is charged
   * every launch it took part in. */
  float ms_filter;       /* window, Chebyshev coefficients and the m filter steps */
  float ms_orth;         /* block Gram-Schmidt against the locked vectors + CholeskyQR2 */
  float ms_rr;           /* Rayleigh-Ritz: A Q, Q^T A Q, eigensolve, rotations */
  float ms_resid;        /* residual norms and locking */
  float ms_bound;        /* upper spectral bound: Gershgorin and the Lanczos run */
  float ms_wall;         /* host wall time from the operator's load to its extraction */
  int32_t magnitude_route; /* SCSF_TARGET_MAGNITUDE: 1 = from the lower end of the spectrum,
                              certified; 2 = with the squared filter; 0 for SCSF_TARGET_SMALLEST */
} scsf_stats;

/* Filter-step timing: when enabled, every Chebyshev step launch of the solvers is bracketed
 * by a pair of HIP events on the handle's stream; the elapsed times and the algorithmic bytes
 * of those launches (read Y_i, Y_{i-1}, write Y_{i+1}, the operator coefficients once) are
 * accumulated at the solver's existing synchronisation points. */
typedef struct scsf_profile {
  int64_t filter_launches;
  double filter_ms;
  double filter_bytes;
  /* Device time per step of Algorithm 3 (filter, orthonormalisation, Rayleigh-Ritz,
   * residuals + locking, bounds) of every outer iteration of the solvers, summed over the
   * lanes; recorded whether or not filter timing is enabled. */
  double phase_ms[5];
} scsf_profile;

/* Handle on the current HIP device, enqueueing on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  The stream must stay valid while the handle is used. */
int scsf_create(scsf_handle **h, void *hip_stream);
int scsf_destroy(scsf_handle *h);
int scsf_set_stream(scsf_handle *h, void *hip_stream);
const char *scsf_status_string(int status);
/* Library build/version string (host). */
const char *scsf_version(void);
/* Number of lockstep batches the chained solvers (scsf_solve_sequence*, scsf_solve_batched)
 * run concurrently (1..16, default 4; each needs a hardware queue of its own, see
 * GPU_MAX_HW_QUEUES).  Each batch runs on a stream the handle creates (default
 * priority), ordered after the work already enqueued on the handle's stream, and is driven by
 * a host thread of its own; the call returns when every batch has finished. */
int scsf_set_lanes(scsf_handle *h, int lanes);
/* The plain FP64 filter of the grid stencils (STENCIL5, STENCIL9) in groups of `steps`
 * Chebyshev steps per launch (2, 3 or 4; 0 = one step per launch, the default): each launch
 * stages the two newest levels of a tile of nodes with its halo in LDS, runs the steps there
 * and writes the last two levels, so a group of S steps moves 4 instead of 3 S block columns
 * through HBM (the same recurrence of Algorithm 1, node by node; results agree to rounding).
 * A degree below S, mixed precision, adaptive degrees,
 * the squared filter, CSR and thin-plate operators keep one step per launch; per-problem
 * degrees (hints) are raised by at most 2 S - 1 so that every problem ends with a whole group.
 * SCSF_EINVAL for another value. */
int scsf_set_fused_steps(scsf_handle *h, int steps);
/* Chained solvers: on != 0 (default) replays each outer iteration of Algorithm 3 as three HIP
 * graphs captured once per filter degree (window and coefficients; the filter's m steps;
 * orthonormalisation, Rayleigh-Ritz, residuals and locking); on == 0 launches the same
 * kernels one by one.  Results are identical either way. */
int scsf_set_graphs(scsf_handle *h, int on);
/* The eigensolver of the Rayleigh-Ritz step (the reduced problem G W = W Theta of
 * Algorithm 3): SCSF_EIG_JACOBI (default: parallel cyclic Jacobi, sweeping until the largest
 * relative off-diagonal entry is at most tol / 100, within [1e-14, 1e-10]; the warm-started
 * projected matrices are nearly diagonal, so one or two sweeps usually suffice) or
 * SCSF_EIG_TRIDIAG (Householder tridiagonalisation, Sturm bisection and inverse iteration: a
 * fixed amount of work).  Both return the eigenvalues ascending with orthonormal
 * eigenvectors. */
int scsf_set_eigensolver(scsf_handle *h, int which);
/* Turn filter-step timing on (on != 0) or off; synchronises the stream. */
int scsf_profile_enable(scsf_handle *h, int on);
/* Copy the accumulated filter timing to *out_host; reset != 0 clears it afterwards. */
int scsf_profile_read(scsf_handle *h, scsf_profile *out_host, int reset);

/* ---------------------------------------------------------------------------------------
 * Device workspace.  By default the handle allocates its device buffers itself (hipMalloc,
 * grown on demand and kept until scsf_destroy).  A caller that owns device memory gives it to
 * the handle instead; from then on the library allocates no device memory of its own: every
 * entry point carves its buffers from that area (256-byte aligned, from its base again at the
 * start of each call, since no device buffer outlives a call) and returns SCSF_ENOMEM, with
 * nothing enqueued, when the area is too small.  The HIP runtime's own objects (streams,
 * events, graph executables of the chained solvers) are created by the runtime.  The
 * solves' inputs follow Algorithm 3's I/O (the operator, the previous subspace, the degree)
 * and their outputs stay in caller memory.
 * ------------------------------------------------------------------------------------- */

/* Device bytes scsf_solve needs for one operator of dimension n with parameters p. */
int scsf_workspace_bytes(const scsf_params *p, int64_t n, size_t *bytes);
/* Device bytes scsf_solve_sequence (hinted = 0) or scsf_solve_sequence_hinted (hinted != 0)
 * needs for n_op operators of dimension n in `chains` chains, with the handle's current lane
 * count (scsf_set_lanes), the up-front bounds of the n_op operators included. */
int scsf_workspace_bytes_sequence(scsf_handle *h, const scsf_params *p, int64_t n, int32_t n_op,
                                  int32_t chains, int32_t hinted, size_t *bytes);
/* Hand the handle `bytes` bytes of device memory at dev_ptr (256-byte aligned) as its only
 * device workspace; the buffers it allocated before are freed (the handle's streams are
 * synchronised first).  dev_ptr = NULL returns to library-allocated buffers.  The caller keeps
 * ownership and must keep the memory valid until the workspace is replaced or the handle is
 * destroyed.  SCSF_EINVAL for a misaligned pointer or a zero size. */
int scsf_set_workspace(scsf_handle *h, void *dev_ptr, size_t bytes);
/* The largest number of workspace bytes any call used since scsf_set_workspace. */
int scsf_workspace_peak(scsf_handle *h, size_t *bytes);

/* ---------------------------------------------------------------------------------------
 * Step primitives of the hot path.  Each is a building block of scsf_solve, exposed so the
 * steps can be checked one by one.
 * ------------------------------------------------------------------------------------- */

/* Y = A X for ncols columns (n x ncols blocks, leading dimensions ldx, ldy). */
int scsf_spmm(scsf_handle *h, const scsf_operator *A, const double *X, int64_t ldx,
              int32_t ncols, double *Y, int64_t ldy);

/* Chebyshev filter, Algorithm 1 with the scaled three-term recurrence (Section 2.2):
 * Y = C_m((A - cI)/e) X / C_m((lambda - c)/e), degree m >= 1, e > 0, lambda != c.
 * X is not modified.  ncols <= 256. */
int scsf_filter(scsf_handle *h, const scsf_operator *A, const double *X, int64_t ldx,
                int32_t ncols, int32_t degree, double lambda, double c, double e,
                double *Y, int64_t ldy);

/* The filter of Algorithm 1 on B blocks at once, one per operator, in the lockstep form the
 * chained solvers use (every Chebyshev step is one launch over all B blocks):
 * Y_b = C_m((A_b - c_b I)/e_b) X_b / C_m((lambda_b - c_b)/e_b), b = 0..B-1.
 * ops_host: B operators of one kind (host array of device-backed descriptors); sizes may differ.
 * X, Y: device; block b at X + b*bsx (Y + b*bsy), n_b rows, ncols columns, column-major with
 * leading dimension ldx (ldy) >= max n_b, bsx >= ldx*ncols, bsy >= ldy*ncols.  The two block
 * ranges must not overlap; X is not modified.  win_host: host, (lambda_b, c_b, e_b) per block,
 * e_b > 0, lambda_b != c_b.  ncols <= 256, degree 1..128.  The steps use the handle's filter
 * tile (scsf_set_tile, scsf_autotune); while profiling is on (scsf_profile_enable) every step
 * launch is timed with a pair of HIP events on the caller's stream and counted with its
 * algorithmic bytes.  Synchronises the stream.  SCSF_EINVAL on invalid arguments. */
int scsf_filter_batched(scsf_handle *h, const scsf_operator *ops_host, int32_t B,
                        const double *X, int64_t ldx, int64_t bsx, int32_t ncols, int32_t degree,
                        const double *win_host, double *Y, int64_t ldy, int64_t bsy);

/* Gram matrices of B blocks at once, G_b = X_b^T X_b (the first product of CholeskyQR2,
 * Algorithm 3): the solvers' tall-skinny MFMA kernel (f64 16x16x4) with its deterministic
 * chunk reduction.  X: device, block b at X + b*bsx, n x k column-major, ldx >= n,
 * bsx >= ldx*k, k <= 256.  G: device, block b at G + b*ldg*k, k x k column-major (both
 * triangles), ldg >= k.  kernel_ms_host: when non-NULL, receives the time of the Gram kernels
 * alone (HIP events on the caller's stream).  Synchronises the stream. */
int scsf_gram_batched(scsf_handle *h, int32_t B, int64_t n, int32_t k, const double *X,
                      int64_t ldx, int64_t bsx, double *G, int32_t ldg, double *kernel_ms_host);

/* Orthonormalisation of Algorithm 3 (QR of [locked | active]): X (n x ncols, in place) is
 * made orthogonal to the nlocked orthonormal columns V (twice-repeated block Gram-Schmidt),
 * then orthonormalised by CholeskyQR2 (shifted CholeskyQR3 if the Gram matrix is not
 * numerically positive definite).  V may be NULL when nlocked = 0.  ncols + nlocked <= 256. */
int scsf_orthonormalize(scsf_handle *h, int64_t n, double *X, int64_t ldx, int32_t ncols,
                        const double *V, int64_t ldv, int32_t nlocked);

/* Rayleigh-Ritz and residuals (Algorithm 3, Rayleigh quotient + reduced eigenproblem +
 * residual check): for orthonormal X (n x ncols, in place) forms G = X^T A X, solves
 * G W = W Theta (ascending), sets X <- X W, and writes theta[ncols] and the relative residuals
 * rel_resid[j] = ||A x_j - theta_j x_j|| / ||A x_j||.  ncols <= 256. */
int scsf_rayleigh_ritz(scsf_handle *h, const scsf_operator *A, double *X, int64_t ldx,
                       int32_t ncols, double *theta, double *rel_resid);

/* Upper spectral bound for the filter window: out_host[0] = Gershgorin bound,
 * out_host[1] = theta_max(T_s) + beta_s of an s-step Lanczos run from a seeded random start,
 * out_host[2] = theta_min(T_s), out_host[3] = min(out_host[0], out_host[1]). */
int scsf_bounds(scsf_handle *h, const scsf_operator *A, int32_t steps, uint64_t seed,
                double *out_host);

/* scsf_bounds without any device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernel and outputs as scsf_bounds, with its scratch (the operator descriptor, the
 * three Lanczos vectors and the bounds) in a fixed 8 MiB device array of the library, which
 * each GPU holds from the first scsf_create on it until the process ends.  n <= 262144
 * (SCSF_EINVAL above); SCSF_EHIP if the array's device address could not be obtained.  No
 * hipMalloc, hipFree or other allocating call is made.  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (from several handles or threads) race.  Synchronises
 * the handle's stream. */
int scsf_bounds_noalloc(scsf_handle *h, const scsf_operator *A, int32_t steps, uint64_t seed,
                        double *out_host);

/* Truncated-FFT features of Algorithm 2: for each of n_op fields (channels x p x p real,
 * row-major, contiguous per operator) the p0 x p0 corner k1, k2 in [0, p0) of the 2-D DFT
 * divided by p^2.  feats: n_op x channels x p0 x p0 complex (re, im interleaved). */
int scsf_features(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels,
                  int32_t p, int32_t p0, double *feats);

/* Algorithm 2 end to end: order_host[n_op] = greedy nearest-neighbour order of the
 * truncated-FFT features, starting at `start`; ties go to the lowest index.  p0 <= p.
 * A NaN or infinite distance (non-finite fields, or squared differences that overflow) ranks
 * as +infinity, so order_host is still a permutation, but the call returns SCSF_EINVAL. */
int scsf_sort(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels,
              int32_t p, int32_t p0, int32_t start, int32_t *order_host);

/* The greedy nearest-neighbour order of Algorithm 2 on precomputed features: feats (device)
 * holds n_op rows of flen complex numbers (re, im interleaved), e.g. scsf_features outputs of
 * fields of different sides p concatenated (the 1/p^2 scaling makes them comparable).
 * Squared Frobenius distances; ties go to the lowest index.  n_op <= 32768; needs n_op^2
 * doubles of workspace.  Non-finite distances: as scsf_sort (SCSF_EINVAL). */
int scsf_order_features(scsf_handle *h, const double *feats, int32_t n_op, int32_t flen,
                        int32_t start, int32_t *order_host);

/* Sort diagnostics (App. F; the appendix on the truncation threshold p0).
 *
 * scsf_highfreq_ratio: for each operator, ||F_high||_F / ||F||_F over its channels, where F is
 * the 2-D DFT of each p x p field and F_high holds the coefficients whose signed frequency
 * (index a read as a for a <= p/2, a - p above) is >= p0 in absolute value on either axis.
 * fields: device, (n_op, channels, p, p) row-major; ratio: device, n_op doubles.  A field
 * that is zero everywhere gives 0.  Synchronises the handle's stream.
 *
 * The full greedy order of Section 3.1 (no truncation) is scsf_order_features on the raw
 * fields (flen = channels * p * p): the spatial Frobenius distance.
 *
 * scsf_subspace_distance: the one-sided distance ||(I - U U^T) V||_2 (the sine of the largest
 * principal angle) between the spans of the first q columns of blocks a_host[i] and b_host[i]
 * of X, i = 0..P-1; the columns must be orthonormal (eigenvectors from the solvers).  X:
 * device, n_blocks blocks at stride bsx, each n x (>= q) column-major with leading dimension
 * ldx >= n, bsx >= ldx * q; 1 <= q <= min(32, n).  out_host: host, P doubles.  SCSF_EINVAL on
 * an index outside [0, n_blocks) or another invalid argument. */
int scsf_highfreq_ratio(scsf_handle *h, const double *fields, int32_t n_op, int32_t channels,
                        int32_t p, int32_t p0, double *ratio);
int scsf_subspace_distance(scsf_handle *h, int64_t n, int32_t q, const double *X, int64_t ldx,
                           int64_t bsx, int32_t n_blocks, const int32_t *a_host,
                           const int32_t *b_host, int32_t P, double *out_host);

/* ---------------------------------------------------------------------------------------
 * Solvers.
 * ------------------------------------------------------------------------------------- */

/* One operator, Algorithm 3.  X_prev (n x k, ld n) and theta_prev (k) are the previous
 * problem's Ritz pairs (warm start) or both NULL (cold start from a seeded Gaussian block).
 * Outputs: evals[L] ascending (by |lambda| with SCSF_TARGET_MAGNITUDE; M-orthonormal u for
 * SCSF_PLATE), evecs (n x L, ld n; largest-magnitude entry positive),
 * X_next (n x k, ld n) and theta_next[k] for chaining (may alias X_prev / theta_prev).
 * stats_host may be NULL. */
int scsf_solve(scsf_handle *h, const scsf_operator *A, const scsf_params *prm,
               const double *X_prev, const double *theta_prev, double *evals, double *evecs,
               double *X_next, double *theta_next, scsf_stats *stats_host);

/* A whole dataset (Fig. 2 c-d): ops_host[n_op] (host array of operator descriptors, all of
 * the same kind and n) are solved in the order order_host[n_op] split into `chains`
 * contiguous chunks (App. D.6 chunking); the chunks run concurrently (lockstep batches on
 * up to scsf_set_lanes streams), each chain warm-starting every solve from its previous one.
 * The spectral bound of every operator (the scsf_bounds run, its Lanczos start vector keyed by
 * the operator's index) is computed up front in batched launches before the chains start.
 * evals: n_op x L (row i = operator i), evecs: n_op x (n x L) (block i = operator i, ld n).
 * stats_host[n_op] may be NULL.  Returns SCSF_ENOTCONV if any solve did not converge. */
int scsf_solve_sequence(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                        const int32_t *order_host, int32_t chains, const scsf_params *prm,
                        double *evals, double *evecs, scsf_stats *stats_host);

/* The learned-window form: as scsf_solve_sequence, with per-operator hints_host[n_op*3] =
 * (predicted lambda_1, predicted lambda_{L+1}, predicted degree) in operator index order.
 * A positive degree replaces prm->degree for that operator (1..128, clamped to 64 with
 * SCSF_MIXED; within a lockstep batch
 * degrees are raised by at most 2 to a common residue mod 3).  The predicted window replaces
 * the Ritz-value window of the operator's first outer iteration if the Lanczos bounds accept it:
 * lambda_1 <= theta_min(T_s) and lambda_1 < lambda_{L+1} < beta (stats.hint reports 2 / 3);
 * otherwise the plain window is used.  hints_host may be NULL.  ritz (device, n_op x k, may be
 * NULL) receives every operator's k final Ritz values, ascending (the labels of the window
 * network). */
int scsf_solve_sequence_hinted(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                               const int32_t *order_host, int32_t chains,
                               const scsf_params *prm, const double *hints_host, double *evals,
                               double *evecs, double *ritz, scsf_stats *stats_host);

/* ---------------------------------------------------------------------------------------
 * Uneven batches (operators of different sizes and different L in one call).  Not in the
 * paper: its chunked dataset runs (App. D.6) generalised to mixed sizes.
 * ------------------------------------------------------------------------------------- */

/* Default block width k for L wanted pairs: the smallest multiple of 8 that is >= L plus
 * ceil(0.2 L) guard vectors (at most 256).  SCSF_EINVAL unless 0 < L < 256. */
int scsf_block_width(int32_t L);

/* Autotuner (project-specific; the paper fixes its block widths by hand, Section 4).  For
 * every distinct L of the dataset (ops_host / L_host / order_host as in scsf_solve_batched):
 *  - tiles: the LDS-staged filter step is timed with 1, 2 and 4 block columns per thread (and
 *    8, 4, 2 grid nodes per thread) on 8 to 64 copies (a working set of about 768 MB) of the
 *    largest operator of each size bucket (n <= 4096, <= 16384, larger) for each width
 *    bucket (k <= 48, <= 96, <= 160, larger) it meets; another tile replaces the default 4
 *    only when it is at least 10% faster;
 *  - widths: the first `probe` operators of the L group (in order_host order) are solved as
 *    one warm-started chain with block widths 1.2 L, 1.35 L and 1.5 L (rounded up to a
 *    multiple of 8, at most 256 and at most the smallest n), and the width with the least
 *    time wins (a width whose probe does not converge never wins).
 * The results stay in the handle: scsf_solve_batched with k_host == NULL uses the tuned
 * width, and every chained solve uses the tuned tile for its (n, k).  prm as in
 * scsf_solve_batched; 1 <= probe <= 64.  Runs synchronously; allocates its probe outputs. */
int scsf_autotune(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                  const int32_t *L_host, const int32_t *order_host, const scsf_params *prm,
                  int32_t probe);
/* The tuned block width for L (scsf_block_width(L) when L was never tuned). */
int scsf_tuned_width(scsf_handle *h, int32_t L);
/* Set the filter-step tile (block columns per thread of the LDS-staged step: 1, 2, 4 or 8,
 * with 8 / tile nodes per thread) for every size and width, overriding the autotuner (which
 * chooses among 1, 2 and 4); the fused and thin-plate steps take at most 4.  SCSF_EINVAL for
 * another value. */
int scsf_set_tile(scsf_handle *h, int32_t tile);
/* The tuned filter-step tile (block columns per thread: 1, 2 or 4; default 4) for size n and
 * width k. */
int scsf_tuned_tile(scsf_handle *h, int64_t n, int32_t k);

/* Bilinear transfer of ncols nodal fields between interior grids of the unit square: column
 * c of X (device, N0*N0 entries, node (iy, ix) at entry iy*N0 + ix, ld ldx >= N0^2) is read as
 * a field with zero Dirichlet boundary and evaluated at the N1 x N1 nodes into column c of Y
 * (device, ld ldy >= N1^2).  X and Y must not overlap (SCSF_EINVAL).  Used to warm-start a
 * solve from the Ritz vectors of an operator on a grid of another side. */
int scsf_interpolate(scsf_handle *h, int32_t N0, int32_t N1, int32_t ncols, const double *X,
                     int64_t ldx, double *Y, int64_t ldy);

/* A dataset of operators of different sizes and different numbers of wanted pairs.
 * ops_host[n_op]: descriptors (any mix of sizes; kinds may differ).  L_host[n_op]: wanted
 * pairs per operator (0 < L < 256).  k_host[n_op]: block widths, or NULL for the
 * autotuned width of each L (scsf_tuned_width).  prm supplies degree, tol, max_iter,
 * lanczos_steps, seed, schedule, precision (SCSF_MIXED: the FP32 filter of the sequence
 * solvers; not for SCSF_PLATE) and target (prm->L and prm->k are ignored).
 * The operators are grouped by (kind, L, k), keeping order_host's order inside each group,
 * and every group is split into chains (about chains * group size / n_op of them) that run as
 * in scsf_solve_sequence (per group, or all groups of a kind in one batch: scsf_set_batch_form).  Along a chain each solve warm-starts from the previous one; when
 * the grid side changes the Ritz vectors are moved by scsf_interpolate's transfer (operators
 * not on square grids restart cold).
 * Outputs, packed in operator-index order: evals[sum L_i] with operator i at
 * sum_{j<i} L_j, evecs[sum n_i L_i] with operator i's n_i x L_i block (ld n_i) at
 * sum_{j<i} n_j L_j.  stats_host[n_op] may be NULL.  Returns SCSF_ENOTCONV if any solve did
 * not converge. */
/* The form of scsf_solve_batched's lockstep batches (the outer iteration of Algorithm 3 over
 * the chunks of App. D.6; batching operators of different sizes is not in the paper).
 * SCSF_BATCH_GROUPED (default): each
 * (kind, L, k) group runs as its own batches (a lane starts at its own group and takes the
 * others in turn).  SCSF_BATCH_ONE_SWEEP: every lane runs one batch over the chains of all
 * groups of a kind, so each sweep (outer iteration of Algorithm 3) covers operators of every
 * (L, k) in the same launches and graphs.  There, each problem occupies the last k_i columns
 * of a block as wide as the widest group: the columns before them are zero and locked from
 * the start, and every step of the iteration works on a problem's active columns only.  Not
 * with adaptive degrees or SCSF_TARGET_MAGNITUDE (those solves return SCSF_EINVAL).  Results
 * agree with the grouped form to the solves' tolerance (the random first blocks differ).
 * SCSF_EINVAL for another value. */
int scsf_set_batch_form(scsf_handle *h, int form);
int scsf_solve_batched(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                       const int32_t *L_host, const int32_t *k_host, const int32_t *order_host,
                       int32_t chains, const scsf_params *prm, double *evals, double *evecs,
                       scsf_stats *stats_host);
/* scsf_solve_batched with per-operator window and degree hints, hints_host[n_op*3] in
 * operator index order, as in scsf_solve_sequence_hinted (the learned-window form on uneven
 * batches; SCSF_EINVAL with adaptive degrees or SCSF_TARGET_MAGNITUDE).  hints_host may be
 * NULL. */
int scsf_solve_batched_hinted(scsf_handle *h, const scsf_operator *ops_host, int32_t n_op,
                              const int32_t *L_host, const int32_t *k_host,
                              const int32_t *order_host, int32_t chains,
                              const scsf_params *prm, const double *hints_host, double *evals,
                              double *evecs, scsf_stats *stats_host);

/* ---------------------------------------------------------------------------------------
 * Spectral-window network (the learned form of the window of Section 2.2; not in the paper).
 * Input: the truncated-FFT features of Algorithm 2 with 3 channels and p0 = 16, fed as 6 real
 * channels (Re, Im).  Layers: conv 3x3 6->16 stride 1 + ReLU, conv 3x3 16->32 stride 2 + ReLU,
 * dense 2048->64 + ReLU, dense 64->3 (zero padding 1).  Parameters: one flat FP32 device array
 * W1[16,6,3,3] b1[16] W2[32,16,3,3] b2[32] W3[64,2048] b3[64] W4[3,64] b4[3].
 * Outputs: (log lambda_1, log lambda_{L+1}, degree / 128).
 * ------------------------------------------------------------------------------------- */

/* Number of FP32 parameters. */
int scsf_window_param_count(void);
/* He-normal weights (Philox keyed by seed), zero biases. */
int scsf_window_init(scsf_handle *h, float *params, uint64_t seed);
/* feats: n x 3 x 16 x 16 complex (re, im) from scsf_features -> x: n x 6 x 16 x 16 FP32. */
int scsf_window_input(scsf_handle *h, const double *feats, int32_t n, int32_t channels,
                      int32_t p0, float *x);
/* out[n*3] = network(x); bf16 != 0 stores parameters and activations in BF16 (FP32 sums). */
int scsf_window_forward(scsf_handle *h, const float *params, const float *x, int32_t n,
                        int32_t bf16, float *out);
/* FP32 loss mean((y - t)^2)/2 and its gradient (device, param_count floats). */
int scsf_window_loss_grad(scsf_handle *h, const float *params, const float *x,
                          const float *target, int32_t n, float *grad, double *loss_host);
/* Full-batch Adam (lr, betas 0.9 / 0.999) for `epochs` steps from zero moments; params in place;
 * loss_history_host[epochs] may be NULL. */
int scsf_window_train(scsf_handle *h, float *params, const float *x, const float *target,
                      int32_t n, int32_t epochs, float lr, double *loss_history_host);
/* Training targets from solved operators: ritz (n x k ascending), beta[n] (the upper bounds
 * used) -> target[n*3] = (log lambda_1, log lambda_{L+1}, mstar / 64) with
 * mstar = clamp(ceil(acosh(1e4) / acosh|t(lambda_L)|), 8, 128) over the damped [lambda_{L+1}, beta]. */
int scsf_window_labels(scsf_handle *h, const double *ritz, int32_t n, int32_t k, int32_t L,
                       const double *beta, float *target);
/* hints[n*3] (device, for scsf_solve_sequence_hinted) = (exp y0, exp y1, round(128 y2) clamped
 * to [8, 128]). */
int scsf_window_hints(scsf_handle *h, const float *out, int32_t n, double *hints);

#ifdef __cplusplus
}
#endif
#endif /* SCSF_H */
