// Preconditioner factorizations for the Cholesky route.
//
//  * Gram matrix of the sketch, C = Z^T Z (Algorithm 1 step 3 with Z = Y,
//    Algorithm 2 step 3 with Z = Y^T).
//  * For every lambda of a batch, R = chol(C + lambda I) (upper triangular,
//    R^T R = C + lambda I; Algorithm 1 step 4, Algorithm 2 step 4), then the
//    explicit inverse R^{-1}.  LSQR applies R^{-1} and R^{-T} many times; as
//    explicit triangular matrices each application is one fully parallel
//    matrix-vector product instead of a sequential substitution.  The solve
//    only needs R^{-1} to be a fixed nonsingular matrix: LSQR returns
//    x = R^{-1} y* for the y* that is optimal for that very matrix, so the
//    computed inverse's rounding changes the convergence rate, not x.
//
// Blocked right-looking factorization with 64 x 64 blocks, batched over the
// lambdas (grid.y = matrix): per block column a diagonal factor+invert kernel
// in LDS, a panel kernel and a trailing update; then the inverse is assembled
// block column by block column, Rinv[0:l, l] = -Rinv[0:l, 0:l] R[0:l, l] D_l
// with D_l the inverse of the diagonal block.  Breakdown (a pivot that is not
// positive and finite) is flagged per lambda; the paper assumes it cannot
// happen when kappa(C + lambda I) < O(1/u) (Section 2.1.1).
#include "tik_internal.h"

namespace tik {

static constexpr int NB = 64;

// ------------------------------------------------- 64 x 64 FP64 MFMA tiles --
// acc += op(A) B for one 64 x 64 output tile on the matrix cores
// (v_mfma_f64_16x16x4_f64).  op(A) is 64 x K: A itself (TA = false, element
// (i, k) at A[i + k lda]) or the transpose of a K x 64 block (TA = true,
// element (i, k) at A[k + i lda]); B is K x 64 (element (k, j) at
// B[k + j ldb], or at B[j + k ldb] with TB).  Rows >= mrows, columns >= ncols and k >= K read as zero.
// Wave w owns the 32 x 32 quarter (rows 32 (w & 1), columns 32 (w >> 1)) as
// 2 x 2 MFMA tiles; K is staged through LDS 32 at a time.  Result element
// (row 32 (w & 1) + 16 t + 4 v + lane / 16, column 32 (w >> 1) + 16 u +
// lane % 16) is acc[t][u][v].
typedef double f64x4 __attribute__((ext_vector_type(4)));
static constexpr int TK = 32;

struct TileLds {
  double As[64][TK + 1];
  double Bs[TK][64 + 1];
};

// DEPTH 1: the next chunk of K is fetched into registers while the matrix
// cores use the current one from LDS.  DEPTH 2: two register sets take turns,
// so the chunk after next is in flight as well; the few-chunk contractions of
// the panel solve, the trailing update and the inverse's last step run faster
// that way (it also leaves the compiler fewer live values: 72 VGPRs instead of
// 142 for the trailing update), while the long contractions of k_trinv_mul
// keep DEPTH 1 (with two sets they drop to one block per CU).
template <bool TA, int DEPTH = 1, bool TB = false>
__device__ __forceinline__ void tile_mma(const double* __restrict__ A, int64_t lda,
                                         const double* __restrict__ B, int64_t ldb, int64_t K,
                                         int mrows, int ncols, TileLds& L, f64x4 (&acc)[2][2]) {
  static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = 32 * (wv & 1), wc = 32 * (wv >> 1);
  constexpr int Q = 64 * TK / 256;     // elements of each tile per thread
  auto fetch = [&](int64_t k0, double (&ra)[Q], double (&rb)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (TA) { kk = e % TK; i = e / TK; } else { i = e % 64; kk = e / 64; }
      const int64_t k = k0 + kk;
      double v = 0.0;
      if (i < mrows && k < K) v = TA ? A[k + int64_t(i) * lda] : A[i + k * lda];
      ra[q] = v;
      int kb, j;
      if (TB) { j = e % 64; kb = e / 64; } else { kb = e % TK; j = e / TK; }
      const int64_t kg = k0 + kb;
      rb[q] = (j < ncols && kg < K) ? (TB ? B[j + kg * ldb] : B[kg + int64_t(j) * ldb]) : 0.0;
    }
  };
  auto stash = [&](const double (&ra)[Q], const double (&rb)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      if (TA) L.As[e / TK][e % TK] = ra[q];
      else L.As[e % 64][e / 64] = ra[q];
      if (TB) L.Bs[e / 64][e % 64] = rb[q];
      else L.Bs[e % TK][e / TK] = rb[q];
    }
  };
  auto mma = [&]() {
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = L.As[wr + 16 * t + li][kk + lk];
#pragma unroll
      for (int u = 0; u < 2; ++u) b[u] = L.Bs[kk + lk][wc + 16 * u + li];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
  };
  double ra0[Q], rb0[Q];
  if (K > 0) {
    fetch(0, ra0, rb0);
    stash(ra0, rb0);
  }
  if constexpr (DEPTH == 1) {
    __syncthreads();
    for (int64_t k0 = 0; k0 < K; k0 += TK) {
      const bool more = k0 + TK < K;
      if (more) fetch(k0 + TK, ra0, rb0);
      mma();
      __syncthreads();
      if (more) stash(ra0, rb0);
      __syncthreads();
    }
  } else {
    double ra1[Q], rb1[Q];
    if (K > TK) fetch(TK, ra1, rb1);
    __syncthreads();
    // LDS holds chunk k0 and set 1 chunk k0 + TK; K is uniform, so every
    // break is taken by the whole block right after a barrier
    for (int64_t k0 = 0; k0 < K; k0 += 2 * TK) {
      if (k0 + 2 * TK < K) fetch(k0 + 2 * TK, ra0, rb0);
      mma();
      __syncthreads();
      if (k0 + TK >= K) break;
      stash(ra1, rb1);
      __syncthreads();
      if (k0 + 3 * TK < K) fetch(k0 + 3 * TK, ra1, rb1);
      mma();
      __syncthreads();
      if (k0 + 2 * TK >= K) break;
      stash(ra0, rb0);
      __syncthreads();
    }
  }
}

// Visit the tile's elements: f(row, col, value) for the 64 x 64 result.
template <typename F>
__device__ __forceinline__ void tile_for_each(const f64x4 (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = 32 * (wv & 1), wc = 32 * (wv >> 1);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(wr + 16 * t + 4 * v + (lane >> 4), wc + 16 * u + (lane & 15), acc[t][u][v]);
}

__device__ __forceinline__ void tile_zero(f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = f64x4{0, 0, 0, 0};
}

// ---------------------------------------------------------------- Gram ------
// C (n x n, ld n) = Z^T Z with Z K x n column-major (ld ldz), on the matrix
// cores.  Upper tile pairs are computed and written to both triangles.  The
// contraction is split into gridDim.y slices of kc rows of Z: slice 0 writes
// C, slice z > 0 the n x n block P + (z - 1) n^2, and k_gram_sum adds those to
// C in slice order (the few hundred tile pairs of a 2000-column Gram would
// otherwise leave some CUs a third block while most have two).
__global__ void __launch_bounds__(256) k_syrk(const double* __restrict__ Z, int64_t K, int64_t n,
                                              int64_t ldz, double* __restrict__ C,
                                              double* __restrict__ P, int nt, int64_t kc) {
  __shared__ TileLds L;
  // map blockIdx.x to tile pair (ti <= tj)
  int t = blockIdx.x, ti = 0;
  while (t >= nt - ti) { t -= nt - ti; ++ti; }
  const int tj = ti + t;
  const int64_t a0 = int64_t(ti) * 64, b0 = int64_t(tj) * 64;
  const int na = int(min<int64_t>(64, n - a0)), nb = int(min<int64_t>(64, n - b0));
  const int64_t k0 = int64_t(blockIdx.y) * kc, k1 = min(K, k0 + kc);
  double* __restrict__ out = blockIdx.y == 0 ? C : P + int64_t(blockIdx.y - 1) * n * n;
  f64x4 acc[2][2];
  tile_zero(acc);
  tile_mma<true>(Z + k0 + a0 * ldz, ldz, Z + k0 + b0 * ldz, ldz, max<int64_t>(0, k1 - k0), na, nb, L, acc);
  tile_for_each(acc, [&](int i, int j, double v) {
    if (i < na && j < nb) {
      out[(a0 + i) + (b0 + j) * n] = v;
      out[(b0 + j) + (a0 + i) * n] = v;
    }
  });
}

// C += P_0 + P_1 + ... (np blocks of nn values at P), in that order.
__global__ void k_gram_sum(double* __restrict__ C, const double* __restrict__ P, int np, int64_t nn) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nn;
       e += int64_t(gridDim.x) * blockDim.x) {
    double s = C[e];
    for (int z = 0; z < np; ++z) s += P[int64_t(z) * nn + e];
    C[e] = s;
  }
}

// ----------------------------------------------------- shifted copies -------
// The upper triangle (diagonal included) of C + lam I: the factorization reads
// nothing else, and everything below the diagonal is written before it is read
// (diagonal blocks by k_trinv_diag, the inverse's temporaries, k_zero_lower).
__global__ void k_shift_copy(const double* __restrict__ C, int64_t n, const double* __restrict__ lams,
                             double* __restrict__ R) {
  const int64_t mat = blockIdx.y;
  const int64_t nn = n * n;
  double* Rm = R + mat * nn;
  const double lam = lams[mat];
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nn;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    if (r <= c) Rm[e] = C[e] + (r == c ? lam : 0.0);
  }
}

// --------------------------------------------- diagonal block: factor+invert --
// One 64 x 64 diagonal block per matrix.  Thread (ti, tj) = (tid % 16,
// tid / 16) keeps the elements (ti + 16 p, tj + 16 q), p, q < 4, in registers:
// the strided ownership keeps every thread busy while the active corner
// shrinks.  Factorization in the right-looking LDL^T form: at step k the
// owners of row k publish it (double-buffered LDS), one barrier, then every
// thread updates a_ij -= a_ki a_kj / a_kk for k < i <= j; afterwards
// R[i][j] = a_ij / sqrt(a_ii).  The inverse X = R^{-1} by back substitution
// on B = I, last row first: the owners of row k of B publish X[k][.] =
// B[k][.] / R[k][k] and the owners of column k of R publish it, one barrier,
// then B[i][j] -= R[i][k] X[k][j] for i < k <= j.  The step loops are split
// into 4 unrolled blocks of 16 so that the register index is a constant.
// One block per job of the table (jobs whose n <= k0 are finished and return).
// src: the block's input, 64 x 64 with leading dimension 64, in LDS (the
// trailing update that produced it hands it over), or null to read it from R.
__device__ void potrf_diag_block(const CholJob& J, int64_t k0, const double* src) {
  const int64_t n = J.n;
  double* Rm = J.R;
  double* Dinv = J.Dinv;
  const int kb = int(min<int64_t>(NB, n - k0));
  __shared__ double rowb[2][NB];
  __shared__ double colb[2][NB];
  __shared__ double diag[NB];
  __shared__ int bad;
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  double a[4][4], b[4][4];
  if (tid == 0) bad = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, j = tj + 16 * q;
      a[p][q] = (i < kb && j < kb && i <= j) ? (src ? src[i + 64 * j] : Rm[(k0 + i) + (k0 + j) * n])
                                             : 0.0;
      b[p][q] = (i == j && i < kb) ? 1.0 : 0.0;
    }
  // factorization (skipped when the job holds a factor already)
#pragma unroll
  for (int P = 0; P < 4; ++P) {
    if (J.given) break;
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * P + kk;
      if (k >= kb) break;
      const int buf = k & 1;
      if (ti == kk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rowb[buf][tj + 16 * q] = a[P][q];
      }
      __syncthreads();
      double d = rowb[buf][k];
      if (!(d > 0.0) || !isfinite(d)) d = 1.0;     // flagged below; keeps the rest finite
      const double inv = 1.0 / d;
      double ri[4], rj[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) ri[p] = rowb[buf][ti + 16 * p] * inv;
#pragma unroll
      for (int q = 0; q < 4; ++q) rj[q] = rowb[buf][tj + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti + 16 * p, j = tj + 16 * q;
          if (i > k && i <= j && j < kb) a[p][q] -= ri[p] * rj[q];
        }
    }
  }
  // pivots: sqrt(a_ii), breakdown flag (a given factor: its own diagonal)
  if (ti == tj) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = ti + 16 * p;
      if (i < kb) {
        double d = a[p][p];
        if (J.given) {
          if (!(d != 0.0) || !isfinite(d)) {
            bad = 1;
            d = 1.0;
          }
          diag[i] = d;
        } else {
          const double fl = J.dg ? J.floor * J.dg[k0 + i] : 0.0;
          if (!(d > fl) || !isfinite(d)) {
            bad = 1;
            d = 1.0;
          }
          diag[i] = sqrt(d);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, j = tj + 16 * q;
      double v = 0.0;
      if (i < kb && j < kb && i <= j) v = J.given ? a[p][q] : ((i == j) ? diag[i] : a[p][q] / diag[i]);
      a[p][q] = v;
      if (i < kb && j < kb) Rm[(k0 + i) + (k0 + j) * n] = v;
    }
  // inverse
#pragma unroll
  for (int P = 3; P >= 0; --P) {
    for (int kk = 15; kk >= 0; --kk) {
      const int k = 16 * P + kk;
      if (k >= kb || k == 0) continue;
      const int buf = k & 1;
      if (ti == kk) {
        const double rk = 1.0 / diag[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) rowb[buf][tj + 16 * q] = b[P][q] * rk;
      }
      if (tj == kk) {
#pragma unroll
        for (int p = 0; p < 4; ++p) colb[buf][ti + 16 * p] = a[p][P];
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti + 16 * p, j = tj + 16 * q;
          if (i < k && j >= k && j < kb) b[p][q] -= colb[buf][i] * rowb[buf][j];
        }
    }
  }
  double* D = Dinv + (k0 / NB) * NB * NB;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, j = tj + 16 * q;
      D[i + j * NB] = (i < kb && j < kb && i <= j) ? b[p][q] / diag[i] : 0.0;
    }
  __syncthreads();
  if (tid == 0 && bad) *J.notpd = 1;
}

__global__ void __launch_bounds__(256) k_potrf_diag(const CholJob* __restrict__ jobs, int64_t k0) {
  const CholJob J = jobs[blockIdx.x];
  if (k0 >= J.n) return;                     // uniform
  potrf_diag_block(J, k0, nullptr);
}

// R[k0:k0+kb, cols] = D^T R[k0:k0+kb, cols] for the 64-column tile blockIdx.x
// right of the diagonal block (D = inverse of the diagonal block).  In place:
// the tile is read completely before it is written.
__global__ void __launch_bounds__(256) k_trsm_panel(const CholJob* __restrict__ jobs, int64_t k0) {
  __shared__ TileLds L;
  const CholJob J = jobs[blockIdx.y];
  const int64_t n = J.n;
  double* Rm = J.R;
  const int kb = int(min<int64_t>(NB, n - k0));
  const int64_t c0 = k0 + kb + int64_t(blockIdx.x) * 64;
  if (k0 >= n || c0 >= n) return;           // uniform: no such tile in this job
  const int nc = int(min<int64_t>(64, n - c0));
  const double* Dm = J.Dinv + (k0 / NB) * NB * NB;
  f64x4 acc[2][2];
  tile_zero(acc);
  tile_mma<true, 2>(Dm, NB, Rm + k0 + c0 * n, n, kb, kb, nc, L, acc);
  tile_for_each(acc, [&](int i, int c, double v) {
    if (i < kb && c < nc) Rm[(k0 + i) + (c0 + c) * n] = v;
  });
}

// Trailing update of the upper tiles: R[a, b] -= R[k, a]^T R[k, b] over the
// KW panel rows k from k0 (tile pair a <= b, tiles counted from k0 + KW), or
// with ROW_ONLY over the first tile row only (a = 0).
// Tile 0 of each job updates the next diagonal block and then factors and
// inverts it (the diagonal step of the next panel, from the updated values it
// keeps in LDS): launched first, it runs beside the other tiles' updates
// instead of in a launch of its own after them.
// The 128-row contraction prefetches one K chunk ahead and runs three blocks
// per CU (two chunks ahead, or four blocks per CU, spill its registers).
template <int KW, bool ROW_ONLY>
__global__ void __launch_bounds__(256, KW == 64 ? 4 : 3)
    k_syrk_trail(const CholJob* __restrict__ jobs, int64_t k0) {
  __shared__ TileLds L;
  // blocks in dispatch order take tile 0 of every job first, then tile 1, ...:
  // the diagonal steps start before the other tiles, not one job at a time
  const int64_t lin = int64_t(blockIdx.x) + int64_t(blockIdx.y) * gridDim.x;
  const int tile = int(lin / gridDim.y);
  const CholJob J = jobs[lin % gridDim.y];
  const int64_t n = J.n;
  double* Rm = J.R;
  if (k0 >= n) return;                       // uniform
  const int kb = int(min<int64_t>(KW, n - k0));
  const int nt = int(cdiv(n - k0 - kb, 64));    // this job's trailing tiles
  if (tile >= (ROW_ONLY ? nt : nt * (nt + 1) / 2)) return;   // uniform
  int t = tile, ta = 0;
  if (!ROW_ONLY)
    while (t >= nt - ta) { t -= nt - ta; ++ta; }
  const int tb = ta + t;
  const int64_t base = k0 + kb;
  const int64_t a0 = base + int64_t(ta) * 64, b0 = base + int64_t(tb) * 64;
  const int na = int(min<int64_t>(64, n - a0)), nb = int(min<int64_t>(64, n - b0));
  f64x4 acc[2][2];
  tile_zero(acc);
  tile_mma<true, KW == 64 ? 2 : 1>(Rm + k0 + a0 * n, n, Rm + k0 + b0 * n, n, kb, na, nb, L, acc);
  if (tile != 0) {
    tile_for_each(acc, [&](int i, int j, double v) {
      if (i < na && j < nb) Rm[(a0 + i) + (b0 + j) * n] -= v;
    });
    return;
  }
  // the next diagonal block: tile_mma ended on a barrier, so its LDS is free
  static_assert(sizeof(TileLds) >= 64 * 64 * sizeof(double), "diagonal block in the tile's LDS");
  double* dblk = reinterpret_cast<double*>(&L);
  tile_for_each(acc, [&](int i, int j, double v) {
    if (i < na && j < nb) {
      const double nv = Rm[(a0 + i) + (b0 + j) * n] - v;
      Rm[(a0 + i) + (b0 + j) * n] = nv;
      dblk[i + 64 * j] = nv;
    }
  });
  __syncthreads();
  potrf_diag_block(J, a0, dblk);
}

// Triangular inverse by recursive doubling, in place.  With the diagonal
// blocks of size s already inverted, each pair of neighbouring blocks A =
// [A0, A0 + s), B = [A0 + s, A0 + 2 s) gets its off-diagonal block
//   Rinv[A, B] = -Rinv[A, A] (R[A, B] Rinv[B, B])
// in two launches over every pair and job: T = R[A, B] Rinv[B, B], kept
// transposed in the strict lower triangle (rows B, columns A: free space), then
// Rinv[A, B] = -Rinv[A, A] T over R[A, B].  Starting from the 64 x 64 inverses
// of the diagonal step, log2(n / 64) levels give R^{-1}; the lower triangle is
// cleared at the end.  Every level is a batch of 64 x 64 MFMA tiles over all
// jobs, instead of one narrow launch per 64-column block.

// Level start: each 64 x 64 diagonal block of R becomes its inverse D_l, with
// zeros below its diagonal (contractions over a diagonal block read them).
__global__ void __launch_bounds__(256) k_trinv_diag(const CholJob* __restrict__ jobs) {
  const CholJob J = jobs[blockIdx.y];
  const int64_t n = J.n;
  const int64_t l0 = int64_t(blockIdx.x) * NB;
  if (l0 >= n) return;                       // uniform
  const int lb = int(min<int64_t>(NB, n - l0));
  const double* Dm = J.Dinv + (l0 / NB) * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e & 63, c = e >> 6;
    if (i < lb && c < lb) J.R[(l0 + i) + (l0 + c) * n] = (i <= c) ? Dm[i + c * NB] : 0.0;
  }
}

// pair and tile of a level's launch, in an order that dispatches the longest
// contractions first: for T (contraction over 64 (tj + 1) rows) the tiles of a
// pair run by descending tj, for Rinv[A, B] (over s - 64 ti rows) by ascending ti
struct LvlTile {
  int64_t a0, b0;
  int ti, tj, bsz;
  bool ok;
};
__device__ __forceinline__ LvlTile lvl_tile(int64_t tile, int64_t n, int64_t s, bool tj_major) {
  const int64_t w = s / 64, per = w * w;
  const int64_t p = tile / per, r = tile % per;
  LvlTile t;
  t.a0 = 2 * s * p;
  t.b0 = t.a0 + s;
  t.ti = int(tj_major ? r % w : r / w);
  t.tj = int(tj_major ? w - 1 - r / w : r % w);
  t.bsz = int(min<int64_t>(s, n - t.b0));
  t.ok = t.b0 < n && 64 * t.tj < t.bsz;
  return t;
}

// T = R[A, B] Rinv[B, B] for tile (ti, tj), stored transposed at rows B,
// columns A.  Rinv[B, B] is upper triangular, so the contraction stops at the
// tile's last column.
__global__ void __launch_bounds__(256) k_trinv_lvl_t(const CholJob* __restrict__ jobs, int64_t s) {
  __shared__ TileLds L;
  // the jobs' tiles interleaved in dispatch order, so the longest of every job go first
  const int64_t lin = int64_t(blockIdx.x) + int64_t(blockIdx.y) * gridDim.x;
  const CholJob J = jobs[lin % gridDim.y];
  const int64_t n = J.n;
  const LvlTile t = lvl_tile(lin / gridDim.y, n, s, true);
  if (!t.ok) return;                         // uniform
  double* Rm = J.R;
  const int64_t r0 = t.a0 + 64 * t.ti, c0 = t.b0 + 64 * t.tj;
  const int nc = int(min<int64_t>(64, t.bsz - 64 * t.tj));
  const int64_t K = min<int64_t>(t.bsz, 64 * (t.tj + 1));
  f64x4 acc[2][2];
  tile_zero(acc);
  tile_mma<false, 1>(Rm + r0 + t.b0 * n, n, Rm + t.b0 + c0 * n, n, K, 64, nc, L, acc);
  tile_for_each(acc, [&](int i, int c, double v) {
    if (c < nc) Rm[(c0 + c) + (r0 + i) * n] = v;
  });
}

// Rinv[A, B] = -Rinv[A, A] T for tile (ti, tj); Rinv[A, A] is upper
// triangular, so the contraction starts at the tile's first row.
__global__ void __launch_bounds__(256, 4) k_trinv_lvl_x(const CholJob* __restrict__ jobs, int64_t s) {
  __shared__ TileLds L;
  const int64_t lin = int64_t(blockIdx.x) + int64_t(blockIdx.y) * gridDim.x;
  const CholJob J = jobs[lin % gridDim.y];
  const int64_t n = J.n;
  const LvlTile t = lvl_tile(lin / gridDim.y, n, s, false);
  if (!t.ok) return;                         // uniform
  double* Rm = J.R;
  const int64_t r0 = t.a0 + 64 * t.ti, c0 = t.b0 + 64 * t.tj;
  const int nc = int(min<int64_t>(64, t.bsz - 64 * t.tj));
  const int64_t K = s - 64 * t.ti;
  f64x4 acc[2][2];
  tile_zero(acc);
  // T(k, j) of this tile sits at Rm[(c0 + j) + (r0 + k) n]
  tile_mma<false, 1, true>(Rm + r0 + r0 * n, n, Rm + c0 + r0 * n, n, K, 64, nc, L, acc);
  tile_for_each(acc, [&](int i, int c, double v) {
    if (c < nc) Rm[(r0 + i) + (c0 + c) * n] = -v;
  });
}

// Clear the strict lower triangle (the level temporaries and whatever the
// factorization's diagonal tiles left below the diagonal).
__global__ void __launch_bounds__(256) k_zero_lower(const CholJob* __restrict__ jobs) {
  const CholJob J = jobs[blockIdx.y];
  const int64_t n = J.n;
  const int64_t c = blockIdx.x;
  if (c >= n) return;                        // uniform
  for (int64_t i = c + 1 + threadIdx.x; i < n; i += 256) J.R[i + c * n] = 0.0;
}

// Column absolute sums of the symmetric Gram matrix C (k x k): their maximum
// bounds ||C||_2 from above (Gershgorin), which bounds kappa(B)^2 by
// (||C|| + lambda) / lambda for the sketched B = [XA; sqrt(lambda) I].
__global__ void __launch_bounds__(256) k_col_abs_sum(const double* __restrict__ C, int64_t n,
                                                     double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += fabs(C[r + c * n]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_max_reduce(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s = fmax(s, v[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

int launch_gram_norm_bound(const double* C, int64_t n, double* scratch, double* out,
                           hipStream_t st) {
  ProfScope ps("gram", st);
  hipLaunchKernelGGL(k_col_abs_sum, dim3(unsigned(n)), dim3(256), 0, st, C, n, scratch);
  TIK_LAUNCHED("k_col_abs_sum");
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, st, scratch, n, out);
  TIK_LAUNCHED("k_max_reduce");
  return TIK_OK;
}

// ---------------------------------------------------------------- launchers --
int launch_syrk(const double* Z, int64_t K, int64_t n, int64_t ldz, double* C, double* P, int maxp,
                hipStream_t st) {
  const int nt = int(cdiv(n, 64));
  const int64_t pairs = int64_t(nt) * (nt + 1) / 2;
  ProfScope ps("gram", st);
  // slices: about eight blocks per CU in all, each slice at least 512 rows of Z
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 0;
  int64_t ks = 1;
  if (P && maxp > 0 && cus > 0) {
    const int64_t hi = std::max<int64_t>(1, std::min<int64_t>(1 + maxp, K / 512));
    ks = std::min<int64_t>(hi, std::max<int64_t>(1, cdiv(8 * int64_t(cus), pairs)));
  }
  const int64_t kc = cdiv(std::max<int64_t>(K, 1), ks);
  ks = cdiv(std::max<int64_t>(K, 1), kc);          // no empty slice
  hipLaunchKernelGGL(k_syrk, dim3(unsigned(pairs), unsigned(ks)), dim3(256), 0, st, Z, K, n, ldz, C, P,
                     nt, kc);
  TIK_LAUNCHED("k_syrk");
  if (ks > 1) {
    const int64_t nn = n * n;
    hipLaunchKernelGGL(k_gram_sum, dim3(unsigned(std::min<int64_t>(cdiv(nn, 256), 4096))), dim3(256), 0,
                       st, C, static_cast<const double*>(P), int(ks - 1), nn);
    TIK_LAUNCHED("k_gram_sum");
  }
  return TIK_OK;
}

int launch_shift_copy(const double* C, int64_t n, const double* lams, int32_t nb_mat, double* R,
                      hipStream_t st) {
  ProfScope ps("chol", st);
  const unsigned gx = unsigned(std::min<int64_t>(cdiv(n * n, 256), 4096));
  hipLaunchKernelGGL(k_shift_copy, dim3(gx, unsigned(nb_mat)), dim3(256), 0, st, C, n, lams, R);
  TIK_LAUNCHED("k_shift_copy");
  return TIK_OK;
}

// Blocked right-looking Cholesky of every job, then the blocked inverse, one
// launch per kernel and panel for the whole table: panel kb covers the jobs
// with n > kb NB (a prefix, the table being sorted by n), each grid sized for
// the largest of them; blocks beyond a smaller job's tiles return at once.
__global__ void k_save_diag(const CholJob* __restrict__ jobs) {
  const CholJob J = jobs[blockIdx.y];
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (J.dg && c < J.n) J.dg[c] = J.R[c + c * J.n];
}

int launch_save_diag(const CholJob* jobs, int32_t njobs, int64_t nmax, hipStream_t st) {
  if (njobs <= 0) return TIK_OK;
  hipLaunchKernelGGL(k_save_diag, dim3(unsigned(cdiv(nmax, 256)), unsigned(njobs)), dim3(256), 0, st,
                     jobs);
  TIK_LAUNCHED("k_save_diag");
  return TIK_OK;
}

int launch_chol_inv_jobs(const CholJob* jobs, const int64_t* nsz, int32_t njobs, hipStream_t st,
                         bool given) {
  if (njobs <= 0) return TIK_OK;
  const int64_t nmax = nsz[0];
  const int64_t nblk = cdiv(nmax, NB);
  auto active = [&](int64_t k0) {            // jobs with n > k0
    int32_t c = 0;
    while (c < njobs && nsz[c] > k0) ++c;
    return c;
  };
  {
    ProfScope ps("chol", st);
    if (given) {
      // triangular factors already: only the diagonal blocks' inverses
      for (int64_t kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(k_potrf_diag, dim3(unsigned(active(kb * NB))), dim3(256), 0, st, jobs, kb * NB);
        TIK_LAUNCHED("k_potrf_diag");
      }
    } else {
      // Two 64-column panels per step: panel k0 is solved and applied to the
      // next tile row only (which factors the next diagonal block), panel
      // k0 + 64 is solved, and both update the rest of the trailing matrix in
      // one pass with 128 contraction rows, so each trailing tile is read and
      // written once per 128 columns instead of once per 64.
      hipLaunchKernelGGL(k_potrf_diag, dim3(unsigned(active(0))), dim3(256), 0, st, jobs, int64_t(0));
      TIK_LAUNCHED("k_potrf_diag");
      for (int64_t k0 = 0; k0 < nmax; k0 += 2 * NB) {
        const int64_t rest1 = nmax - k0 - std::min<int64_t>(NB, nmax - k0);
        if (rest1 <= 0) break;
        const int32_t nr1 = active(k0 + NB);
        const int nt1 = int(cdiv(rest1, 64));
        hipLaunchKernelGGL(k_trsm_panel, dim3(unsigned(nt1), unsigned(nr1)), dim3(256), 0, st, jobs, k0);
        TIK_LAUNCHED("k_trsm_panel");
        hipLaunchKernelGGL((k_syrk_trail<NB, true>), dim3(unsigned(nt1), unsigned(nr1)), dim3(256), 0, st,
                           jobs, k0);
        TIK_LAUNCHED("k_syrk_trail");
        const int64_t rest2 = nmax - k0 - 2 * NB;
        if (rest2 <= 0) break;
        const int32_t nr2 = active(k0 + 2 * NB);
        const int nt2 = int(cdiv(rest2, 64));
        hipLaunchKernelGGL(k_trsm_panel, dim3(unsigned(nt2), unsigned(nr2)), dim3(256), 0, st, jobs,
                           k0 + NB);
        TIK_LAUNCHED("k_trsm_panel");
        hipLaunchKernelGGL((k_syrk_trail<2 * NB, false>), dim3(unsigned(nt2 * (nt2 + 1) / 2), unsigned(nr2)),
                           dim3(256), 0, st, jobs, k0);
        TIK_LAUNCHED("k_syrk_trail");
      }
    }
  }
  {
    ProfScope ps("trinv", st);
    hipLaunchKernelGGL(k_trinv_diag, dim3(unsigned(nblk), unsigned(njobs)), dim3(256), 0, st, jobs);
    TIK_LAUNCHED("k_trinv_diag");
    for (int64_t s = NB; s < nmax; s *= 2) {
      const int32_t na = active(s);          // jobs with a pair at this level
      const int64_t pairs = cdiv(nmax - s, 2 * s);
      const dim3 grid(unsigned(pairs * (s / 64) * (s / 64)), unsigned(na));
      hipLaunchKernelGGL(k_trinv_lvl_t, grid, dim3(256), 0, st, jobs, s);
      TIK_LAUNCHED("k_trinv_lvl_t");
      hipLaunchKernelGGL(k_trinv_lvl_x, grid, dim3(256), 0, st, jobs, s);
      TIK_LAUNCHED("k_trinv_lvl_x");
    }
    hipLaunchKernelGGL(k_zero_lower, dim3(unsigned(nmax), unsigned(njobs)), dim3(256), 0, st, jobs);
    TIK_LAUNCHED("k_zero_lower");
  }
  return TIK_OK;
}

}  // namespace tik
