// Internal declarations shared by the libtik translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/tik.h"

namespace tik {

// ------------------------------------------------------------------ errors --
void set_error(const std::string& msg);

#define TIK_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::tik::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return TIK_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define TIK_LAUNCHED(what)                                                         \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) {                                                        \
      ::tik::set_error(std::string("launch of ") + (what) + ": " + hipGetErrorString(e_)); \
      return TIK_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define TIK_TRY(expr)                 \
  do {                                \
    int rc_ = (expr);                 \
    if (rc_ != TIK_OK) return rc_;    \
  } while (0)

// --------------------------------------------------------------- profiling --
// Records HIP events around each launch of a kernel family when enabled.
struct ProfScope {
  ProfScope(const char* family, hipStream_t st);
  ~ProfScope();
  int slot;
  hipStream_t st;
};
// Forget the last launch recorded for a family: a launch whose kernels
// returned at once (the surplus iteration of a solve loop) moved no data.
void prof_drop_last(const char* family);
// Whether per-launch events are being recorded (the solve loops then launch
// each iteration's kernels directly instead of replaying a captured graph).
bool prof_active();

// True inside tik_lsqr_batch_static: the solve loop then allocates nothing
// (no pinned host words, events or graphs) and waits once per iteration.
bool noalloc_active();

// ----------------------------------------------------------------- options --
// Iterations per graph-captured chunk of the solve loops (0: no graphs).
int option_chunk();
// A Cholesky pivot d_j counts as a breakdown when d_j <= ulps * 2^-53 * (the
// j-th diagonal entry of C + lambda I); 0: only non-positive pivots.
int64_t option_pivot_ulps();
// Nonzeros per column of the sparse embedding (1..16).
int option_sparse_nnz();
// 1: the Householder QRs of the low-rank route and of the QR fallback factor
// each 32-column panel by two Cholesky QR passes and a reconstruction of its
// reflectors, falling back to one launch per column where the panel's scaled
// Gram matrix is nearly singular; 0: one launch per column always.
int option_cholqr_panels();
// 1: SRHT sketches use the column-resident transform where it applies (0: the
// two-pass transform everywhere).
int option_srht_cols();
// 1: the last, partly filled round of the A W product's row blocks is computed
// as column pieces over the whole GPU (single-problem plans); 0: whole blocks.
int option_gemm_n_tail();

// --------------------------------------------------------------- workspace --
// Bump allocator over a caller-provided device buffer.  With base == nullptr it
// only measures, which is how the *_bytes queries are answered.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T) + 0;
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ device structs --
// One problem as the solve kernels see it.  "long" rows are the m rows of a
// tall problem (the n columns of a wide one); "short" rows the other side.
struct DevProb {
  const void* A;
  int64_t m, n, lda;
  int32_t a_f32;
  int32_t wide;
  const double* b;
  int64_t offL;        // row offset of this problem inside long-row vector buffers
  int64_t offS;        // row offset inside short-row vector buffers
  int64_t offR;        // offset of vectors indexed by the rows of A (offL tall, offS wide)
  int64_t offC;        // offset of vectors indexed by the columns of A (offS tall, offL wide)
  int64_t cchunk;      // columns of A per chunk of the split A W product (wide problems)
  int32_t nchN;        // number of such chunks (1 for tall problems)
  int32_t pad_;
  int64_t pnOff;       // first row of this problem in the split-product partial buffer
  const double* Rinv;  // upper-triangular inverses, k x k each (k = short dim), col-major,
                       // one per lambda of the problem; a solve uses Rinv + li * k * k
  int64_t k;           // short dimension min(m, n)
  // low-rank route: V (k x s, ld k), S (one row of s per lambda of the
  // problem, zero beyond that lambda's rank), s, and the largest rank smax
  // used by the lambdas of this solve
  const double* V;
  const double* S;
  int64_t s, smax;
  int64_t lrPart;      // offset of this problem in the projection partials (chunks x s x N)
  int64_t lrOpart;     // offset in the expansion partials (column chunks x N x k)
  int64_t lrCoef;      // offset in the scaled projections (smax x N, row-major)
  int64_t lrRch;       // rows of V per projection chunk
  int32_t lrNch;       // projection row chunks
  int32_t lrNjc;       // expansion column chunks in use (ceil(smax / 256))
  // item bookkeeping
  int64_t pnN, pnB, pnQ; // first block of this problem in the partial-norm arrays
  int32_t nblkN, nblkB, nblkQ, nchT;
  int64_t ptOff;       // first row of this problem in the gemm_T partial buffer
  int64_t rchunk;      // rows per gemm_T chunk
  // solves of the plan still active, as counted after the last iteration
  // (null: always run).  The products over A return at once when it reads 0:
  // the solve loop queues one iteration ahead of the count it has seen.
  const int32_t* live;
  // inner solves of the mixed refinement: where this problem's rows sit in
  // the refinement vectors (f, g, dx) and its index there; an inner plan may
  // hold only the problems that still have a lambda to correct
  int64_t irL, irS;
  int32_t gp, pad2_;
};

// True once every solve of the plan has stopped (the live word reads 0): the
// kernels of a queued iteration then return at once and leave all state as it
// is.  Uniform over a block, so it may precede barriers.
__device__ __forceinline__ bool plan_stopped(const DevProb& pr) {
  return pr.live && *pr.live == 0;
}

// Per-(problem, lambda) LSQR scalars, all FP64.
struct Scal {
  double lam, sqlam;
  double alpha, beta;       // alpha_i, beta_i of the current step
  double beta_new;          // beta_{i+1} once the u-step is reduced
  double rhobar, phibar;
  double anorm2, bnorm;
  double cx, ce;            // x += cx * e ; e = w - ce * e
  double ialpha, ibeta;     // guarded reciprocals
  double ucoef;             // alpha_i / beta_i, the weight of the old u
  double relres, rnorm, arnorm;
  int32_t active, upd, iters, status;
  int32_t li;               // lambda index inside its problem (selects R^{-1} and the X column)
  int32_t pad1;
  int64_t tstart, tdone;    // device wall clock when the solve loop started and when this solve stopped
};

// item tables: x = problem, y = block index (and z = chunk for gemm_T)
struct Item {
  int32_t p, blk, ch, j;
};

// ------------------------------------------------------------- launchers ----
// sketch (k_sketch.hip)
int launch_srht_rows(uint64_t seed, int k, int64_t s, int32_t* rows, int32_t* bstart, int bbits,
                     hipStream_t st);
int launch_srht_single(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int k,
                       uint64_t seed, const int32_t* rows, int64_t s, double* Y, hipStream_t st);
int launch_srht_twopass(const void* A, int a_f32, int64_t m, int64_t lda, int64_t c0, int64_t nc,
                        int k, int bbits, const int32_t* rows, int64_t s, double* T, double* Y,
                        hipStream_t st);
// Column-resident SRHT (one read of A, no scratch) for m' >= 2^14, at least
// kSrhtColsMinN columns (one workgroup each) and s <= 8192.
constexpr int64_t kSrhtColsMinN = 256;
bool srht_cols_ok(int k, int64_t n, int64_t s);
int launch_srht_cols(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int k, int bbits,
                     const int32_t* rows, int64_t s, double* Y, hipStream_t st);
// X chunk (s rows of kc generated values, row pitch ldx; FP64 needs ldx == kc)
// kind: 0 FP64, 1 BF16, 2 FP16
int launch_gauss_gen(uint64_t seed, int64_t s, int64_t r0, int64_t kc, int64_t ldx, void* Xc,
                     int kind, hipStream_t st);
int launch_sketch_gemm_f64(const double* Xc, int64_t s, int64_t kc, const void* A, int a_f32,
                           int64_t lda, int64_t r0, int64_t ncol, int wide, double* Y,
                           hipStream_t st);
int sketch_bf16_splits(int64_t s, int64_t ncol, int64_t kc, int64_t part_cap);
// 16-bit sketch product: BF16 when cscale is NULL, else FP16 with A's columns
// times cscale (tall problems only)
int launch_sketch_gemm_bf16(const void* Xc, int64_t s, int64_t kc, int64_t ldx, const void* A,
                            int a_f32, int64_t lda, int64_t r0, int64_t ncol, int wide, float* Yacc,
                            int first, float* part, int64_t part_cap, hipStream_t st,
                            const float* cscale = nullptr);
int launch_col_pow2(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, float* cscale,
                    hipStream_t st);
int launch_f32_to_f64_cols(const float* src, double* dst, int64_t s, int64_t ncol, const float* cscale,
                           hipStream_t st);
int launch_f32_to_f64(const float* src, double* dst, int64_t count, hipStream_t st);
// sparse embedding of a tall A (m x n): map holds m * zeta ints; Y s x n (ld s)
int launch_sparse_sketch(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int64_t s,
                         int zeta, uint64_t seed, int32_t* map, double* Y, hipStream_t st);

// factorization (k_factor.hip)
// C = Z^T Z (n x n).  P: room for up to maxp more n x n blocks (or null), where
// the partial products of a split contraction are kept until they are added.
int launch_syrk(const double* Z, int64_t K, int64_t n, int64_t ldz, double* C, double* P, int maxp,
                hipStream_t st);
int launch_gram_norm_bound(const double* C, int64_t n, double* scratch, double* out,
                           hipStream_t st);
// One shifted matrix of the batched Cholesky-inverse: R (n x n, ld n) holds
// C + lambda I on entry and the upper triangle of chol(C + lambda I)^{-1} on
// exit (its strict lower triangle serves as scratch on the way and is zero at
// the end); Dinv (ceil(n / 64) blocks of 64 x 64) holds the inverses of the
// diagonal blocks; *notpd is set to 1 on breakdown.
// given = 1: R already holds an upper-triangular factor (the QR route of a
// breakdown); only its inverse is formed.  dg (n values, or null): the
// diagonal of C + lambda I saved before the factorization; a pivot d_j counts
// as a breakdown when d_j <= floor * dg[j] (floor = 0: only non-positive or
// non-finite pivots).
struct CholJob {
  double* R;
  double* Dinv;
  int32_t* notpd;
  int64_t n;
  double* dg;
  double floor;
  int32_t given, pad_;
};
// R_j <- upper triangle of C + lams[j] I for the nb_mat lambdas of one problem
// (R_j at R + j n^2; below the diagonal R_j is left as it was).
int launch_shift_copy(const double* C, int64_t n, const double* lams, int32_t nb_mat, double* R,
                      hipStream_t st);
// Factor and invert every job of the table (device memory), sorted by n,
// largest first; nsz[i] is the n of job i on the host (same order).
// given: the jobs hold triangular factors already; only invert them.
int launch_chol_inv_jobs(const CholJob* jobs, const int64_t* nsz, int32_t njobs, hipStream_t st,
                         bool given = false);
// dg of every job <- the diagonal of its R (C + lambda I before factoring).
int launch_save_diag(const CholJob* jobs, int32_t njobs, int64_t nmax, hipStream_t st);
// BP2 (Section 4.1): R (k x k, ld k; zeros below the diagonal) from the
// Householder QR of [Y; sqrt(lam) I_k], Y the stored sketch (s x k, ld s).
size_t bp2_scratch_doubles(int64_t s, int64_t k);
int launch_bp2_r(const double* Y, int64_t s, int64_t k, double lam, double* R, double* scratch,
                 hipStream_t st);

// matrix-core products (k_mfma.hip)
// rows: rows of A per gemm_n block (128 or 256); cols: columns per gemm_t block (64 or 128).
// W is in the compute type (float when tc_f32, else double).
// epi 0: u~_top update and norm partials; 1: store A W to out; 2: partial
// products of column chunk it.ch into ut; 3 (128-row blocks): epi 0 for the
// items with j == 0 and, for those with j != 0, epi 2 on descriptor P2 into
// part2, in one launch.
int launch_gemm_n_mfma(int ta_f32, int tc_f32, int nc, int epi, int rows, const DevProb* P,
                       const Item* items, int nitems, int N, const void* W, void* ut,
                       double* out, const Scal* sc, double* pnN, hipStream_t st,
                       const DevProb* P2 = nullptr, void* part2 = nullptr);
// 128-row EPI 0 blocks resident at once on the current device; 0 if unknown.
int gemm_n_resident(int ta_f32, int tc_f32, int nc);
int launch_gemm_t_mfma(int ta_f32, int tc_f32, int u_f64, int nc, int cols, const DevProb* P,
                       const Item* items, int nitems, int N, const void* U, void* part,
                       hipStream_t st);

// low-rank route (k_lowrank.hip)
size_t lowrank_scratch_doubles(int64_t n, int64_t s);
int launch_lowrank_svd(const double* Y, int64_t s, int64_t n, double* V, double* sig,
                       double* scratch, unsigned int* cnt, int32_t* perm, int* sweeps,
                       hipStream_t st);
int launch_lowrank_S(const double* sig, int64_t s, const double* lams, const int32_t* si, int N,
                     double* S, hipStream_t st);
struct LrItems {      // device item tables of the low-rank apply and their lengths
  const Item *P, *C, *E, *F;
  int nP, nC, nE, nF;
};
struct LrBufs {       // projection partials, scaled projections, expansion partials
  double *part, *coef, *opart;
};
int launch_lr_apply(int nc, int stage, int tall, const DevProb* P, const LrItems& it, int N,
                    const double* src, const LrBufs& lb, double* q, double* v, double* w, double* x,
                    double* e, const Scal* sc, double* pn, int init, hipStream_t st);
// L-curve norms (k_lcurve.hip)
int lcurve_bytes(const tik_problem* p, int32_t nprob, size_t* bytes);
int lcurve_run(const tik_problem* p, int32_t nprob, int32_t N, double* const* X, double* xnorm,
               double* rnorm, void* dws, size_t dws_bytes, hipStream_t st);
}  // namespace tik

// ----------------------------------------------------------------- handles --
struct tik_sketch_s {
  std::vector<tik_problem> probs;
  int32_t embed = 0, sketch_dtype = 0;
  std::vector<int64_t> s;
  uint64_t seed = 0;
  bool wide = false;
  std::vector<double*> Y;              // per problem: yrows x ycols, column-major, ld = yrows
  std::vector<int64_t> yrows, ycols;   // tall: s x n (Y); wide: s x m (Y^T)
};

struct tik_precond_s {
  std::vector<tik_problem> probs;
  bool wide = false;
  int32_t route = 0, N = 0;
  std::vector<double> lams;            // nprob * N, host copy
  std::vector<int64_t> k;              // short dimension per problem
  std::vector<double*> Rinv;           // Cholesky route: N upper-triangular k x k inverses
  std::vector<int32_t> status;         // nprob * N breakdown flags (tik_status)
  std::vector<uint8_t> qr;             // nprob * N: R came from the QR fallback
  std::vector<double> cnorm;           // per problem: upper bound on ||C||_2 of the sketch Gram
  // low-rank route: V k x s (ld k), sigma (s), S (N x s), truncation s_i
  std::vector<double*> V, sigma, S;
  std::vector<int64_t> srank;
  std::vector<int32_t> si;             // nprob * N
  std::vector<double> sdhat;           // nprob * N
  std::vector<int32_t> lr_sweeps;      // Jacobi sweeps the SVD took, per problem
};

namespace tik {
// split of the last solve on this thread (fp32-refined, fp64) lambdas
void note_split(int32_t fp32, int32_t fp64);
// Completion times of the last tik_lsqr_batch call of this thread (option
// "record_times"): after each batched group's loop, the group's scalars are
// read back and, for every (problem k, lambda i) it solved, (tdone - tstart
// of the call's first group) in ms is stored at k * N + i.
bool option_record_times();
void times_reset(int64_t count);
void times_note(const Scal* host_sc, int J, int N, const std::vector<int>& pidx, const std::vector<int>& lsel,
                int Ntot, hipStream_t st);
void last_split(int32_t* fp32, int32_t* fp64);
// solve driver (k_lsqr.hip)
int lsqr_bytes(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode,
               size_t* bytes);
int lsqr_run(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode,
             double tol, int32_t maxit, double* const* X, int32_t* iters, int32_t* status,
             double* relres, void* dws, size_t dws_bytes, hipStream_t st);
// launch-shape tuning (k_lsqr.hip)
int tune_bytes(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, size_t* bytes);
int tune_class(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t iters, void* dws,
               size_t dws_bytes, hipStream_t st, int* best, double* best_ms, double* default_ms);
int tiles_save(const char* path);
int tiles_load(const char* path, int* loaded);
const std::string& last_tile();
}  // namespace tik
