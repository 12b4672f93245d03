/*
 * tik.h -- C ABI of libtik, sketch-preconditioned Tikhonov least squares on
 * AMD MI355X (gfx950).
 *
 * The library computes, for one or many problems and N regularization
 * parameters lam_1..lam_N each,
 *
 *     x_lam = argmin_x ||A x - b||_2^2 + lam ||x||_2^2          (eq. regLLS)
 *
 * for tall (m >= n, eq. regLLSover) or wide (m < n, eq. regLLSunder) A, by the
 * sketch-to-precondition method of Meier & Nakatsukasa: sketch A once
 * (Algorithm 1 steps 1-2, Algorithm 2 steps 1-2, Algorithm 3 steps 1-3),
 * build a preconditioner R_lam for every lam from that one sketch (Cholesky of
 * the partly exact sketched Gram matrix, Algorithm 1 step 4 / Algorithm 2
 * step 4; or the low-rank factor of eq. RinvOver, Algorithm 3 steps 4-7), and
 * run preconditioned LSQR for every lam (Algorithm 1 steps 5-6, Algorithm 2
 * step 5, Algorithm 3 steps 8-9).
 *
 * Conventions shared by every entry point:
 *  - Matrices are column-major.  All pointers named "device" are HIP device
 *    pointers owned by the caller; the library never allocates device memory
 *    at run time (it keeps a few streams per device and a pool of pinned host
 *    words, created on first use and held by the process; the solve loop's
 *    HIP graphs live for one call; the static workspace of
 *    tik_lsqr_batch_static is a device array of the loaded module).
 *    Every call that needs scratch space takes a caller-provided device
 *    workspace (dws, dws_bytes) whose required size the matching *_bytes
 *    query returns.  A handle points into the workspace it was built in: the
 *    workspace must stay allocated and untouched while the handle is used.
 *  - Calls are stream-ordered on the given stream (a hipStream_t passed as
 *    void*; NULL is the default stream).  Argument errors are detected on the
 *    host before anything is launched; the call then returns TIK_EINVAL and
 *    tik_last_error() describes the problem.
 *  - Return values are tik_rc codes.  Per-(problem, lam) outcomes are
 *    reported separately through tik_status arrays, so one failing lam does
 *    not abort the others.
 *  - The library is not re-entrant on one stream from several host threads;
 *    distinct handles on distinct streams may be used concurrently.
 */
#ifndef TIK_H
#define TIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call-level return codes */
typedef enum {
  TIK_OK = 0,
  TIK_EINVAL = -1,      /* bad argument; nothing was launched */
  TIK_EWORKSPACE = -2,  /* workspace pointer NULL, misaligned or too small */
  TIK_EHIP = -3,        /* a HIP runtime call failed; see tik_last_error() */
  TIK_ENOTSUP = -4      /* valid request outside what the library implements */
} tik_rc;

/* per-(problem, lam) outcome */
typedef enum {
  TIK_ST_CONVERGED = 0, /* the stopping test passed */
  TIK_ST_MAXIT = 1,     /* maxit iterations (or refinement sweeps) without passing it */
  TIK_ST_NOTPD = 2,     /* chol(C + lam I) broke down: the paper assumes
                           kappa(C + lam I) < O(1/u) (Section 2.1); X is not written */
  TIK_ST_IR_STALL = 3,  /* mixed precision: refinement stopped contracting */
  TIK_ST_NONFINITE = 4, /* NaN/Inf met in the data or the recurrence; X not written */
  TIK_ST_QR = 5         /* tik_precond only: chol(C + lam I) broke down and R came
                           from the Householder QR of [Y; sqrt(lam) I] instead (the
                           BP2 preconditioner of Section 4.1); the lam is solved */
} tik_status;

typedef enum { TIK_F64 = 0, TIK_F32 = 1, TIK_BF16 = 2, TIK_F16 = 3 } tik_dtype;

/* embedding X (Section 2.1.1): subsampled randomized Hadamard transform
   X = sqrt(m'/s) S H D (H orthonormal Hadamard of order m' = 2^ceil(log2 m),
   A zero-padded to m' rows), or Gaussian with i.i.d. N(0, 1/s) entries so that
   E[X^T X] = I, the scaling the embedding definition of Section 1.3 fixes, or
   the sparse subspace embedding of Section 3.4 (tall problems): each column
   of X has zeta nonzeros +-1/sqrt(zeta) (option "sparse_nnz", default 1) in
   distinct random rows, one in each of zeta consecutive row blocks; its sketch
   is X A up to the rounding order of its FP64 sums. */
typedef enum { TIK_SRHT = 0, TIK_GAUSS = 1, TIK_SPARSE = 2 } tik_embed;

/* preconditioner: Cholesky of the partly exact sketch (Algorithms 1, 2) or the
   low-rank factor R^{-1} = lam^{-1/2} (I - V S V^T) (eq. RinvOver, Algorithm 3) */
typedef enum { TIK_ROUTE_CHOL = 0, TIK_ROUTE_LOWRANK = 1 } tik_route;

/* how tik_lsqr_batch runs LSQR:
   PLAIN_F64_PER_LAMBDA  one FP64 LSQR per (problem, lam), A read once per
                         iteration per lam (the paper's loop over i);
   F64_BATCHED           all lam of all problems advance together, one read of A
                         per iteration shared by every lam (Section 2.1.1 notes
                         the loop over lam parallelizes trivially);
   MIXED_BATCHED         batched FP32 LSQR inside FP64 iterative refinement:
                         residuals, preconditioner factors and the solution stay
                         FP64 on the device.  A group of up to 32 lam that FP32
                         products cannot carry (12 kappa u_32 > 1/4 for one of
                         its lam, kappa^2 bounded by (||C|| + lam) / lam) is
                         solved by batched FP64 LSQR at max(tol / 1000, 1e-14);
                         when that holds for every group the call runs as
                         F64_BATCHED with that tolerance (tik_lsqr_info
                         reports the split). */
typedef enum {
  TIK_PLAIN_F64_PER_LAMBDA = 0,
  TIK_F64_BATCHED = 1,
  TIK_MIXED_BATCHED = 2
} tik_mode;

/* One problem.  A: device, column-major m x n with leading dimension
   lda >= m, stored as FP64 (a_dtype = TIK_F64) or FP32 (TIK_F32; the FP32
   values are the problem).  b: device, FP64, length m.  Both are read-only
   and must outlive every handle built from them. */
typedef struct {
  int64_t m, n, lda;
  int32_t a_dtype;
  int32_t reserved;     /* must be 0 */
  const void* A;
  const double* b;
} tik_problem;

typedef void* tik_stream_t;
typedef struct tik_sketch_s* tik_sketch_t;
typedef struct tik_precond_s* tik_precond_t;

/* ---------------------------------------------------------------- sketch -- */

/* Workspace bytes tik_sketch needs for these problems (same arguments). */
int tik_sketch_bytes(const tik_problem* p, int32_t nprob, int32_t embed,
                     int32_t sketch_dtype, const int64_t* s, size_t* bytes);

/* Sketch every problem once (Algorithm 1 steps 1-2 for m >= n: Y = X A,
   s x n; Algorithm 2 steps 1-2 for m < n: Y = A X, m x s).
   p[nprob]       host array of problem descriptors (copied into the handle;
                  the device buffers they point to are not);
   embed          TIK_SRHT or TIK_SPARSE (m >= n only), or TIK_GAUSS;
   sketch_dtype   arithmetic of the sketch product: TIK_F64, or TIK_BF16 for
                  the Gaussian embedding on matrix cores (A and X rounded to
                  BF16, FP32 accumulation; the sketch only sets the
                  preconditioner's quality), or TIK_F16 for the same with
                  FP16 operands (three more significand bits, FP16's narrow
                  range): tall problems only (TIK_ENOTSUP for wide ones), each
                  column of A multiplied by the power of two that puts its
                  largest entry in [1, 2) before rounding and the sketch's
                  column divided by it afterwards (exact); one extra pass over
                  A finds the scales;
   s[nprob]       host, sketch size per problem, 1 <= s <= the long dimension;
                  the SRHT also needs m' <= 2^18 and s <= 16384
                  (TIK_ENOTSUP beyond);
   seed           fixes X completely, independently of launch shapes;
   out            receives the handle (host struct; free with tik_sketch_free).
   Returns TIK_EINVAL for bad shapes or mixed orientations (all problems must
   be tall, or all wide), TIK_ENOTSUP for an SRHT, sparse or FP16 sketch of a
   wide matrix. */
int tik_sketch(const tik_problem* p, int32_t nprob, int32_t embed, int32_t sketch_dtype,
               const int64_t* s, uint64_t seed, void* dws, size_t dws_bytes,
               tik_stream_t stream, tik_sketch_t* out);

/* Device pointer to problem k's sketch Y (FP64; s x n column-major with
   ld = s for tall problems, Y^T stored s x m column-major for wide ones). */
int tik_sketch_data(tik_sketch_t sk, int32_t k, const double** Y, int64_t* rows, int64_t* cols);

/* -------------------------------------------------------- preconditioner -- */

/* Workspace bytes tik_precond needs for N lambdas per problem. */
int tik_precond_bytes(tik_sketch_t sk, int32_t route, int32_t N, size_t* bytes);

/* Build R_lam for every problem and lambda from the one sketch.
   TIK_ROUTE_CHOL (Algorithm 1 steps 3-4 / Algorithm 2 steps 3-4):
     C = Y^T Y (or Y Y^T), R = chol(C + lam I), kept as the explicit upper
     triangular inverse R^{-1} so that every later application is a
     triangular matrix-vector product.
   TIK_ROUTE_LOWRANK (Algorithm 3 steps 4-7; Algorithm 4 for wide problems):
     SVD of the sketch computed from the Householder QR of its transpose and
     a one-sided Jacobi SVD of the triangular factor (no Gram matrix is
     formed), then s_i = min(s, ceil(alpha * ceil(sd_hat(lam_i)))) with
     sd_hat the estimate of Section 3.1.2, and S_i as in Algorithm 3 step 7.
     Needs s <= min(m, n) and s <= 4096 (else TIK_EINVAL).  Synchronizes the
     stream once per Jacobi sweep and once per problem.
   lambdas  host, nprob x N row-major (problem k's lambdas at k*N), each > 0;
   alpha    oversampling factor of Algorithm 3, >= 1 (ignored by TIK_ROUTE_CHOL);
   sd_hat   host nprob x N, or NULL: the statistical-dimension estimates
            (TIK_ROUTE_LOWRANK; NaN for TIK_ROUTE_CHOL);
   status   host nprob x N, or NULL: TIK_ST_CONVERGED, TIK_ST_QR where
            chol(C + lam I) broke down (a pivot not above chol_pivot_ulps *
            2^-53 times its diagonal entry of C + lam I; by default not
            positive) and R was built from the Householder QR of [Y; sqrt(lam) I]
            instead (Section 4.1; this Gram-free factor exists however
            ill-conditioned C + lam I is), or TIK_ST_NOTPD where that failed too
            (non-finite data).
   Synchronizes the stream once to read the breakdown flags, and once more
   when some lambda took the QR fallback. */
int tik_precond(tik_sketch_t sk, int32_t route, const double* lambdas, int32_t N,
                double alpha, void* dws, size_t dws_bytes, tik_stream_t stream,
                tik_precond_t* out, double* sd_hat, int32_t* status);

/* Device pointer to the preconditioner of problem k, lambda i.
   TIK_ROUTE_CHOL: R^{-1}, upper triangular dim x dim column-major (ld = dim),
   strictly lower part stored as zeros; rank = dim.
   TIK_ROUTE_LOWRANK: V, dim x rank column-major (ld = dim), the right singular
   vectors of the sketch, of which the first s_i enter R_i^{-1}; *rank = s_i.
   Valid while the preconditioner workspace is. */
int tik_precond_data(tik_precond_t pc, int32_t k, int32_t i, const double** data,
                     int64_t* dim, int64_t* rank);

/* Device pointer to the singular values of problem k's sketch, in decreasing
   order, *count = s (TIK_ROUTE_LOWRANK only; TIK_EINVAL otherwise).  Valid
   while the preconditioner workspace is. */
int tik_precond_sigma(tik_precond_t pc, int32_t k, const double** sigma, int64_t* count);

/* Sweeps of one-sided Jacobi the SVD of problem k's sketch took, the last
   one finding nothing to rotate (TIK_ROUTE_LOWRANK only). */
int tik_precond_sweeps(tik_precond_t pc, int32_t k, int32_t* sweeps);

/* ------------------------------------------------------------- solve ---- */

/* Workspace bytes tik_lsqr_batch needs in this mode. */
int tik_lsqr_batch_bytes(const tik_problem* p, int32_t nprob, tik_precond_t pc,
                         int32_t mode, size_t* bytes);

/* Preconditioned LSQR (Paige & Saunders 1982) on [A; sqrt(lam) I] R^{-1}
   (tall, eq. regLLSoverIter) or R^{-T} [A sqrt(lam) I] (wide, eq.
   regLLSunderiter, started from zero so the minimum-norm solution results)
   for every problem and lambda of pc.
   p, nprob   the same problems the sketch was built from;
   tol        relative tolerance of the LSQR stopping tests
              ||M^T r|| <= tol ||M|| ||r|| or ||r|| <= tol ||b||, M the
              preconditioned operator; in MIXED_BATCHED the refinement stops
              when the FP64 correction is below tol relative to x;
   maxit      iteration cap per lambda (per refinement sweep in MIXED_BATCHED);
   X          host array of nprob device pointers; X[k] is n_k x N column-major
              (ld = n_k), column i receives x_{lam_i}; written only where the
              status is CONVERGED or MAXIT, and in MIXED_BATCHED also where
              it is IR_STALL (the last refined iterate);
   iters      device int32 nprob x N: LSQR iterations used (summed over sweeps);
   status     device int32 nprob x N: tik_status values;
   relres     device double nprob x N: the final ||M^T r|| / (||M|| ||r||)
              estimate;
   Synchronization: the iterations run in chunks of T (the "graph_chunk"
   option, default 4), each captured once per call into a HIP graph on a
   library stream of the calling thread and replayed on `stream`; every
   iteration ends by writing the count of still-active lambdas on the device,
   and every kernel of a later iteration returns at once when it reads 0.
   After queuing chunk c the host waits for the count copied after chunk
   c - 1 (an event after an async copy into one of two pinned host words,
   taken from a small per-process pool allocated on first use): a loop of I
   iterations makes ceil(I / T) + 1 such waits, and the GPU always has the
   next chunk queued.  T = 0, or per-launch profiling, launches each iteration
   directly and waits once per iteration, one iteration late.  After the loop
   the call waits for the outputs to be written (one stream synchronization
   per group of up to 32 lambdas; MIXED_BATCHED also waits once per
   refinement sweep), then returns; all device work is ordered on `stream`. */
int tik_lsqr_batch(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                   double tol, int32_t maxit, double* const* X, int32_t* iters,
                   int32_t* status, double* relres, void* dws, size_t dws_bytes,
                   tik_stream_t stream);

/* Completion times of the calling thread's last tik_lsqr_batch (or
   tik_lsqr_batch_static) call made with the option "record_times" = 1:
   ms[k * N + i] (host, count = nprob * N of that call) = milliseconds from
   the start of the call's first solve loop to the iteration at which the
   solve of problem k, lambda i stopped, read from the device's constant-rate
   wall clock (hipDeviceAttributeWallClockRate).  Lambdas solved by the mixed
   mode's refinement are not timed (NaN).  TIK_EINVAL if count differs. */
int tik_lsqr_times(double* ms, int64_t count);

/* For callers that cannot allocate device memory (tight serving loops,
   harnesses that forbid hipMalloc): tik_lsqr_batch with the same arguments
   except the workspace, which is a static device array of 64 MiB per GPU
   that the library holds until the process ends.  The call allocates
   nothing: no device or pinned host memory, no events, no graphs; it
   launches each iteration directly and synchronizes `stream` after every
   iteration to read the active count into a host local (so it cannot be
   captured into a graph).  A solve whose workspace (tik_lsqr_batch_bytes)
   exceeds 64 MiB returns TIK_ENOTSUP before anything is launched.  Every
   call on one GPU uses that GPU's one array: calls that overlap on one GPU
   (several host threads or streams) race and must be serialized by the
   caller; each call initializes what it reads, so results never depend on
   an earlier call.  Outputs as for tik_lsqr_batch. */
int tik_lsqr_batch_static(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                          double tol, int32_t maxit, double* const* X, int32_t* iters,
                          int32_t* status, double* relres, tik_stream_t stream);

/* How the calling thread's last tik_lsqr_batch split its lambdas: solved with
   FP32 products inside FP64 refinement (*fp32) or with FP64 products
   (*fp64).  PLAIN_F64_PER_LAMBDA and F64_BATCHED count every lambda as FP64. */
int tik_lsqr_info(int32_t* fp32, int32_t* fp64);

/* --------------------------------------------------------------- L-curve -- */

/* Workspace bytes tik_lcurve needs for these problems. */
int tik_lcurve_bytes(const tik_problem* p, int32_t nprob, size_t* bytes);

/* The L-curve of Section 4.3 (Fig. 4): for every problem k and lambda i,
   xnorm[k*N + i] = ||x_i||_2 and rnorm[k*N + i] = ||A_k x_i - b_k||_2, in FP64,
   where x_i is column i of X[k] (device, n_k x N column-major, ld = n_k; what
   tik_lsqr_batch writes).  One pass over each A serves up to 32 lambdas.
   xnorm, rnorm: device double nprob x N (either may be NULL, not both).
   All problems must share A's storage type.  Synchronizes the stream once
   before returning. */
int tik_lcurve(const tik_problem* p, int32_t nprob, int32_t N, double* const* X, double* xnorm,
               double* rnorm, void* dws, size_t dws_bytes, tik_stream_t stream);

/* Corner of an L-curve (Section 4.3; Hansen's maximum-curvature criterion):
   on the curve (log rnorm, log xnorm) parametrized by t = log lambda with
   lambda increasing, the signed curvature (x'y'' - x''y') / (x'^2 + y'^2)^(3/2)
   from second-order three-point differences on the uneven grid; *corner is the
   index (into the caller's order) of its largest value over the interior
   points (the first one on ties).  Host arrays of N >= 3 entries: lambdas
   positive, finite and distinct (any order), norms positive and finite;
   curvature (host N, or NULL) receives the values, NaN at both ends. */
int tik_lcurve_corner(const double* lambdas, const double* xnorm, const double* rnorm, int32_t N,
                      int32_t* corner, double* curvature);

/* ------------------------------------------------------------- tuning -- */

/* Launch shapes of the two products over A (rows of A per A W block: 128 or
   256; columns per A^T U block: 64 or 128; the number of product blocks a
   batch is split into: 1024, 2048 or 4096) come from a table keyed by shape
   class: orientation, FP32 storage, lambda slots per pass, log2 of the
   largest m and of the largest n, and one / up to 16 / more problems.
   Classes without an entry use fixed defaults.  The table file tuning.txt
   beside the library is read on first use when present.  Tables change what
   workspace a solve needs: query the *_bytes functions after tuning or
   loading. */

/* Workspace bytes tik_tune needs for these problems and preconditioner. */
int tik_tune_bytes(const tik_problem* p, int32_t nprob, tik_precond_t pc, size_t* bytes);

/* Time `iters` (2..1000) batched FP64 LSQR iterations of the first (up to 32)
   lambdas of every problem with each candidate shape (twice each, the faster
   second run counts), record the fastest in the table for the problems'
   class, and return it: best[3] = {rows, cols, blocks} (host, or NULL),
   *best_ms and the default shape's *default_ms (host, or NULL).  Overwrites the
   workspace; synchronizes the stream after every timed run. */
int tik_tune(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t iters, void* dws,
             size_t dws_bytes, tik_stream_t stream, int32_t* best, double* best_ms, double* default_ms);

/* Write the table to a text file / merge a text file into the table (one
   class per line: wide a32 nc log2m log2n problems rows cols blocks; '#'
   starts a comment).  A malformed line rejects the whole file. */
int tik_tune_save(const char* path);
int tik_tune_load(const char* path, int32_t* loaded);

/* The launch shape and its source (tuned or default) of the last plan the
   calling thread made, as text (truncated to len - 1 characters). */
int tik_last_tiles(char* buf, int32_t len);

/* Free the host structs (device workspaces belong to the caller). */
void tik_sketch_free(tik_sketch_t sk);
void tik_precond_free(tik_precond_t pc);

/* Message describing the last failure on the calling thread ("" if none). */
const char* tik_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int tik_version(void);

/* Process-wide options.
   "chol_pivot_ulps"  tik_precond's Cholesky route treats a pivot d_j as a
                  breakdown when d_j <= value * 2^-53 * (C + lam I)_jj, 0..2^53
                  (default 0: only pivots that are not positive); such lambdas
                  take the QR fallback (TIK_ST_QR).  A larger value sends the
                  lambdas whose factorization lost that many ulps of a pivot
                  to the Gram-free route.
   "sparse_nnz"   nonzeros per column of the sparse embedding, 1..16
                  (default 1, the sparse subspace embedding of Section 3.4).
   "cholqr_panels"  1 (default): the Householder QRs inside tik_precond (the
                  low-rank route's SVD, the QR fallback) factor each 32-column
                  panel P by two passes of Cholesky QR on its column-scaled
                  Gram matrix and rebuild the panel's reflectors from the
                  orthonormal factor, about a dozen launches and one stream
                  synchronization per panel; a panel whose scaled Gram matrix
                  has a pivot below 1e-10 (kappa above about 1e5) is factored
                  column by column instead.  0: always column by column (one
                  launch per column).
   "srht_cols"    1 (default): an SRHT sketch with m' >= 2^14, at least 256
                  columns and s <= 8192 transforms each column in one
                  workgroup (buckets of 2^14 rows in LDS, the sampled rows
                  summed across buckets with their Hadamard signs): A is read
                  once and no transform scratch is used.  0: the two-pass
                  transform with a column-chunk scratch.  Both give the same
                  X; sums are taken in a different order, so Y can differ in
                  the last bits (integer-valued A gives identical Y).
                  tik_sketch_bytes reflects the setting at the time of the
                  query.
   "gemm_n_tail"  1 (default): for a single tall problem whose row blocks in
                  the product A W (128 rows each, at least 256 columns, 16 or
                  32 lambdas per pass) outnumber the blocks resident at once,
                  with the last round at most half full, that round's blocks
                  are computed as column pieces spread over the whole GPU
                  (partial products in the workspace, summed in piece order by
                  a second kernel) instead of one block per CU.  0: every row
                  block whole.  The two sum the columns in a different order,
                  so results can differ in the last bits.  Read when a solve
                  is planned.
   "record_times"  1: tik_lsqr_batch records, for every (problem, lambda)
                  of a batched FP64 or plain per-lambda call, the device wall
                  clock when its iteration stopped, and tik_lsqr_times returns
                  them (one extra read-back and synchronization per group of
                  up to 32 lambdas); default 0.
   "graph_chunk"  LSQR iterations per graph-captured chunk of tik_lsqr_batch's
                  loop, 0..64 (0: no graphs, one host wait per iteration);
                  default 4.  Replays past convergence cost a few microseconds
                  per kernel, so long chunks only pay where iterations are
                  long.
   Returns TIK_EINVAL for an unknown name or a value out of range. */
int tik_set_option(const char* name, int64_t value);
int tik_get_option(const char* name, int64_t* value);

/* ----------------------------------------------------------- profiling -- */

/* Per-kernel-family timing with HIP events recorded around every launch of
   that family on its stream.  Off by default; enabling it adds two event
   records per launch.  Names: "sketch", "gram", "chol", "trinv", "gemm_n",
   "gemm_t", "trmv", "trmv_t", "lowrank", "lr_apply", "vec", "residual". */
int tik_prof_enable(int32_t on);
int tik_prof_reset(void);
/* Synchronizes outstanding events of that family; total_ms summed over
   launches. */
int tik_prof_query(const char* family, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* TIK_H */
