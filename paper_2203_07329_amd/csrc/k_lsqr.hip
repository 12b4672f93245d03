// Preconditioned LSQR, batched over problems and lambdas (tall problems).
//
// Operator per (problem p, lambda i):  M = [A; sqrt(lam) I] R^{-1}
// (eq. regLLSoverIter, Algorithm 1 step 5, Algorithm 3 step 8).  LSQR is the
// Golub-Kahan bidiagonalisation of Paige & Saunders (1982): for i = 1, 2, ...
//     beta_{i+1} u_{i+1}  = M v_i - alpha_i u_i
//     alpha_{i+1} v_{i+1} = M^T u_{i+1} - beta_{i+1} v_i
// followed by one Givens rotation.  The iterate lives in the preconditioned
// variable y; since only x = R^{-1} y is wanted (Algorithm 1 step 6), the
// search direction is carried already multiplied by R^{-1}: with
// w_i = R^{-1} v_i and e_i = R^{-1} d_i,
//     x_i = x_{i-1} + (phi_i / rho_i) e_i,   e_{i+1} = w_{i+1} - (theta_{i+1}/rho_i) e_i,
// so x comes out in the original variables and no back-transform is needed.
//
// One iteration is eight stream-ordered kernels:
//   gemm_n   u~_top = A w - (alpha/beta) u~_top         one pass over A, all lambdas
//   vec_bot  u~_bot = sqrt(lam) w - (alpha/beta) u~_bot
//   fin_beta beta_{i+1} = ||u~||                         fixed-order reductions
//   gemm_t   partial A^T u~_top over row chunks         one pass over A, all lambdas
//   reduce_t t = (A^T u~_top + sqrt(lam) u~_bot) / beta
//   trmv_t   v~ = R^{-T} t - beta v                     explicit triangular inverse
//   fin_alpha alpha_{i+1} = ||v~||, rotation, stopping tests, masks
//   trmv     w = R^{-1} v~ / alpha, v = v~ / alpha, x and e updates
// All lambdas of all problems share each launch; A is read twice per
// iteration for every lambda together.  Vectors: "long" (m rows) and "short"
// (n rows) buffers are row-major (rows x N, N lambdas per row); t is stored
// lambda-major so the transposed triangular product reads it contiguously.
#include "tik_internal.h"

#include <dlfcn.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace tik {

static constexpr int BLK = 256;

template <typename T>
__device__ __forceinline__ T warp_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block, fixed order.  `red` holds 4 values.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = warp_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Rows per block of the bottom part u~_bot (n rows per problem): small blocks,
// so that the few thousand rows are spread over many compute units.
static constexpr int VB = 32;

// -------------------------------------------------------------- init u -----
// u~ = [rhs_top; rhs_bot] (rhs_top == null: b for every lambda; rhs_bot == null:
// zero) and partial squared norms.  Items: gemm_n blocks (top) then vec_bot
// blocks (bottom), one launch.  Top rows stored in TC.  Thread t handles
// lambda t % N of rows t / N, t / N + BLK / N, ... of the block, and each
// lambda's partial is summed over its threads in a fixed order (one barrier).
template <typename TC>
__global__ void __launch_bounds__(BLK) k_init_u(const DevProb* __restrict__ P,
                                                const Item* __restrict__ itN, int nItN, int rbN,
                                                const Item* __restrict__ itB, int N,
                                                const double* __restrict__ rhs_top,
                                                const double* __restrict__ rhs_bot,
                                                TC* __restrict__ ut, double* __restrict__ ub,
                                                double* __restrict__ pnN, double* __restrict__ pnB) {
  __shared__ double red[BLK];
  const bool top = int(blockIdx.x) < nItN;
  const Item it = top ? itN[blockIdx.x] : itB[blockIdx.x - nItN];
  const DevProb& pr = P[it.p];
  const int64_t rows = top ? pr.m : pr.n;
  const int64_t rb = top ? rbN : VB;
  const int64_t r0 = int64_t(it.blk) * rb;
  const int64_t r1 = min(rows, r0 + rb);
  double* pn = top ? pnN + (pr.pnN + it.blk) * N : pnB + (pr.pnB + it.blk) * N;
  const int rpp = BLK / N;                    // rows per pass
  const int t = threadIdx.x, i = t % N, rr = t / N;
  double loc = 0.0;
  if (rr < rpp) {
    for (int64_t r = r0 + rr; r < r1; r += rpp) {
      double v;
      if (top) {
        v = rhs_top ? rhs_top[(pr.offL + r) * N + i] : pr.b[r];
        const TC vc = TC(v);
        ut[(pr.offL + r) * N + i] = vc;
        v = double(vc);
      } else {
        v = rhs_bot ? rhs_bot[(pr.offS + r) * N + i] : 0.0;
        ub[(pr.offS + r) * N + i] = v;
      }
      loc += v * v;
    }
  }
  red[t] = loc;
  __syncthreads();
  if (t < N) {
    double sum = 0.0;
    for (int j = 0; j < rpp; ++j) sum += red[t + j * N];
    pn[t] = sum;
  }
}

// ------------------------------------------------------------- fin_beta ----
// beta_{i+1} = sqrt(sum of partials).  One block per (problem, lambda).
// pnX, nX: nX more partials of problem 0 (the split A W tail's sub-blocks),
// added after an iteration's product only (init = 0).
__global__ void __launch_bounds__(BLK) k_fin_beta(const DevProb* __restrict__ P, int N,
                                                  const double* __restrict__ pnN,
                                                  const double* __restrict__ pnB,
                                                  Scal* __restrict__ sc, int init,
                                                  const double* __restrict__ pnX, int nX) {
  __shared__ double red[4];
  const int j = blockIdx.x, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  if (plan_stopped(pr)) return;
  double v = 0.0;                             // (unrolled: the loads go out together)
#pragma unroll 4
  for (int b = threadIdx.x; b < pr.nblkN; b += BLK) v += pnN[(pr.pnN + b) * N + i];
  for (int b = threadIdx.x; b < pr.nblkB; b += BLK) v += pnB[(pr.pnB + b) * N + i];
  if (!init && p == 0)
    for (int b = threadIdx.x; b < nX; b += BLK) v += pnX[int64_t(b) * N + i];
  const double s = block_sum(v, red);
  if (threadIdx.x != 0) return;
  Scal& S = sc[j];
  const double beta = sqrt(s);
  S.beta_new = beta;
  S.ibeta = (beta > 0.0 && isfinite(beta)) ? 1.0 / beta : 0.0;
  if (init) {
    S.beta = beta;
    S.bnorm = beta;
    S.phibar = beta;
    if (!isfinite(beta)) {
      S.status = TIK_ST_NONFINITE;
      S.active = 0;
      S.tdone = int64_t(wall_clock64());
    } else if (beta == 0.0) {
      S.status = TIK_ST_CONVERGED;   // b = 0: x = 0
      S.active = 0;
      S.tdone = int64_t(wall_clock64());
    }
  }
}

// --------------------------------------------------------------- gemm_n ----
// u~_top[r, :] = A[r, :] W - ucoef u~_top[r, :] over a block of RB rows;
// EPI = 1 stores the plain product A W into `out` (FP64) instead.
// 256 threads = RB rows x KS column slices; W staged through LDS 64 rows at a
// time (converted to TC); A read column by column, 64..256 consecutive rows
// per wave.
template <typename TA, typename TC, int NC, int RB, int KS, int EPI>
__global__ void __launch_bounds__(BLK) k_gemm_n(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N,
                                                const double* __restrict__ W,
                                                TC* __restrict__ ut, double* __restrict__ out,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ pnN) {
  static_assert(RB * KS == BLK, "block shape");
  constexpr int KC = 64;
  __shared__ TC Ws[KC][NC];
  __shared__ TC red[KS > 1 ? KS : 1][RB][NC > 4 ? 1 : NC];
  __shared__ double nred[4];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (pr.live && *pr.live == 0) return;   // every solve of the plan has stopped
  const TA* __restrict__ A = static_cast<const TA*>(pr.A);
  const int64_t m = pr.m, n = pr.n, lda = pr.lda;
  const int tr = threadIdx.x % RB, ks = threadIdx.x / RB;
  const int64_t r = int64_t(it.blk) * RB + tr;
  const bool live = r < m;
  const int64_t kbeg = int64_t(it.ch) * pr.cchunk;
  const int64_t kend = min(n, kbeg + pr.cchunk);
  TC acc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) acc[i] = TC(0);
  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    const int kc = int(min<int64_t>(KC, kend - k0));
    for (int e = threadIdx.x; e < KC * NC; e += BLK) {
      const int kk = e / NC, i = e % NC;
      Ws[kk][i] = (kk < kc && i < N) ? TC(W[(pr.offC + k0 + kk) * N + i]) : TC(0);
    }
    __syncthreads();
    if (live) {
      const TA* col = A + r + k0 * lda;
      int kk = ks;
      for (; kk + 3 * KS < kc; kk += 4 * KS) {
        const TC a0 = TC(col[int64_t(kk) * lda]);
        const TC a1 = TC(col[int64_t(kk + KS) * lda]);
        const TC a2 = TC(col[int64_t(kk + 2 * KS) * lda]);
        const TC a3 = TC(col[int64_t(kk + 3 * KS) * lda]);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          acc[i] = fma(a0, Ws[kk][i], acc[i]);
          acc[i] = fma(a1, Ws[kk + KS][i], acc[i]);
          acc[i] = fma(a2, Ws[kk + 2 * KS][i], acc[i]);
          acc[i] = fma(a3, Ws[kk + 3 * KS][i], acc[i]);
        }
      }
      for (; kk < kc; kk += KS) {
        const TC a0 = TC(col[int64_t(kk) * lda]);
#pragma unroll
        for (int i = 0; i < NC; ++i) acc[i] = fma(a0, Ws[kk][i], acc[i]);
      }
    }
    __syncthreads();
  }
  if (KS > 1) {
    // combine the KS column slices (only used with NC <= 4)
#pragma unroll
    for (int i = 0; i < (NC > 4 ? 1 : NC); ++i) red[ks][tr][i] = acc[i];
    __syncthreads();
    if (ks == 0) {
#pragma unroll
      for (int i = 0; i < (NC > 4 ? 1 : NC); ++i) {
        TC s = red[0][tr][i];
        for (int q = 1; q < KS; ++q) s += red[q][tr][i];
        acc[i] = s;
      }
    }
  }
  const bool writer = live && ks == 0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    if (i < N) {   // uniform over the block
      double v = 0.0;
      if (writer) {
        if (EPI == 0) {
          const int64_t idx = (pr.offR + r) * N + i;
          const TC nv = TC(acc[i] - TC(sc[it.p * N + i].ucoef) * ut[idx]);
          ut[idx] = nv;
          v = double(nv) * double(nv);
        } else if (EPI == 1) {
          out[(pr.offR + r) * N + i] = double(acc[i]);
        } else {
          ut[(pr.pnOff + int64_t(it.ch) * m + r) * N + i] = acc[i];
        }
      }
      if (EPI == 0) {
        const double s = block_sum(v, nred);
        if (threadIdx.x == 0) pnN[(pr.pnN + it.blk) * N + i] = s;
      }
    }
  }
}

// -------------------------------------------------------------- vec_bot ----
// u~_bot = sqrt(lam) w - ucoef u~_bot and its squared-norm partials for a
// block of VB rows.  Thread t handles lambda t % N of rows t / N, t / N + BLK / N,
// ... (consecutive threads read consecutive lambdas of a row), and the partials
// of a lambda are summed over its threads in a fixed order: one barrier per
// block instead of one reduction per lambda.
__global__ void __launch_bounds__(BLK) k_vec_bot(const DevProb* __restrict__ P,
                                                 const Item* __restrict__ items, int N,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ ub,
                                                 const Scal* __restrict__ sc,
                                                 double* __restrict__ pnB) {
  __shared__ double red[BLK];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int rpp = BLK / N;                    // rows per pass
  const int t = threadIdx.x, i = t % N, rr = t / N;
  const int64_t r0 = int64_t(it.blk) * VB, r1 = min(pr.n, r0 + VB);
  double loc = 0.0;
  if (rr < rpp) {
    const Scal& S = sc[it.p * N + i];
    const double sql = S.sqlam, uc = S.ucoef;
    for (int64_t r = r0 + rr; r < r1; r += rpp) {
      const int64_t idx = (pr.offS + r) * N + i;
      const double nv = sql * w[idx] - uc * ub[idx];
      ub[idx] = nv;
      loc += nv * nv;
    }
  }
  red[t] = loc;
  __syncthreads();
  if (t < N) {
    double s = 0.0;
    for (int j = 0; j < rpp; ++j) s += red[t + j * N];
    pnB[(pr.pnB + it.blk) * N + t] = s;
  }
}

// --------------------------------------------------------------- gemm_t ----
// part[chunk][c][:] = sum over the chunk's rows of A[r, c] U[r, :], for a
// 64-column block.  A and U staged through LDS 32 rows at a time.
//   NC >= 4: thread (column, lambda group of NC/4);
//   NC <  4: thread (column, row slice of 4), slices summed at the end.
template <typename TA, typename TC, typename TU, int NC>
__global__ void __launch_bounds__(BLK) k_gemm_t(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N,
                                                const TU* __restrict__ U, int64_t uoffL_stride,
                                                TC* __restrict__ part) {
  constexpr int RS = 32;
  constexpr int G = NC >= 4 ? NC / 4 : NC;   // accumulators per thread
  __shared__ TC As[RS][64 + 1];
  __shared__ TC Us[RS][NC];
  __shared__ TC red[4][64][NC < 4 ? NC : 1];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (pr.live && *pr.live == 0) return;   // every solve of the plan has stopped
  const TA* __restrict__ A = static_cast<const TA*>(pr.A);
  const int64_t m = pr.m, n = pr.n, lda = pr.lda;
  const int64_t c0 = int64_t(it.blk) * 64;
  const int64_t rbeg = int64_t(it.ch) * pr.rchunk;
  const int64_t rend = min(m, rbeg + pr.rchunk);
  const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
  TC acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = TC(0);
  for (int64_t r0 = rbeg; r0 < rend; r0 += RS) {
    for (int e = threadIdx.x; e < RS * 64; e += BLK) {
      const int rr = e & (RS - 1), cc = e / RS;
      const int64_t rg = r0 + rr, cg = c0 + cc;
      As[rr][cc] = (rg < rend && cg < n) ? TC(A[rg + cg * lda]) : TC(0);
    }
    for (int e = threadIdx.x; e < RS * NC; e += BLK) {
      const int rr = e / NC, i = e % NC;
      const int64_t rg = r0 + rr;
      Us[rr][i] = (rg < rend && i < N) ? TC(U[(pr.offR + rg) * uoffL_stride + i]) : TC(0);
    }
    __syncthreads();
    if (NC >= 4) {
#pragma unroll 8
      for (int rr = 0; rr < RS; ++rr) {
        const TC a = As[rr][cl];
#pragma unroll
        for (int q = 0; q < G; ++q) acc[q] = fma(a, Us[rr][g * G + q], acc[q]);
      }
    } else {
#pragma unroll
      for (int rr = g; rr < RS; rr += 4) {
        const TC a = As[rr][cl];
#pragma unroll
        for (int q = 0; q < G; ++q) acc[q] = fma(a, Us[rr][q], acc[q]);
      }
    }
    __syncthreads();
  }
  const int64_t c = c0 + cl;
  TC* dst = part + (pr.ptOff + int64_t(it.ch) * n) * N;
  if (NC >= 4) {
    if (c < n) {
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int i = g * G + q;
        if (i < N) dst[c * N + i] = acc[q];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < G; ++q) red[g][cl][q] = acc[q];
    __syncthreads();
    if (g == 0 && c < n) {
#pragma unroll
      for (int q = 0; q < G; ++q) {
        if (q < N) dst[c * N + q] = red[0][cl][q] + red[1][cl][q] + red[2][cl][q] + red[3][cl][q];
      }
    }
  }
}

// ------------------------------------------------------------- reduce_t ----
// EPI 0: t[i][c] = (sum_ch part + sqrt(lam) u~_bot[c, i]) / beta, lambda-major.
// EPI 1: out[c, i] = sum_ch part - lam x[c, i] (row-major; FP64 gradient).
// One thread per (row c, lambda i): 256 / NC rows per block.
template <typename TC, int EPI, int NC>
__global__ void __launch_bounds__(BLK) k_reduce_t(const DevProb* __restrict__ P,
                                                  const Item* __restrict__ items, int N,
                                                  const TC* __restrict__ part,
                                                  const double* __restrict__ ub,
                                                  const Scal* __restrict__ sc,
                                                  double* __restrict__ t) {
  constexpr int RR = BLK / NC;
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t n = pr.n;
  const int64_t c = int64_t(it.blk) * RR + threadIdx.x / NC;
  const int i = threadIdx.x % NC;
  if (c >= n || i >= N) return;
  double s = 0.0;
  const TC* src = part + (pr.ptOff + c) * N + i;
  const int64_t stride = n * N;
  int ch = 0;
  for (; ch + 7 < pr.nchT; ch += 8) {      // eight loads in flight, added in chunk order
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = double(src[int64_t(ch + u) * stride]);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += a[u];
  }
  for (; ch < pr.nchT; ++ch) s += double(src[int64_t(ch) * stride]);
  const Scal& S = sc[it.p * N + i];
  if (EPI == 0) {
    t[pr.offS * N + int64_t(i) * n + c] = (s + S.sqlam * ub[(pr.offS + c) * N + i]) * S.ibeta;
  } else {
    t[(pr.offS + c) * N + i] = s - S.lam * ub[(pr.offS + c) * N + i];
  }
}

// --------------------------------------------------------------- trmv_t ----
// v~[c] = sum_{r <= c} Rinv[r, c] t[r] - beta v[c] for a block of 4 * CPW
// columns of one (problem, lambda); each wave owns CPW columns, lanes stride
// the rows (coalesced along the columns of Rinv and along t).
// WIDE (Algorithm 2, R^{-T} applied on the u side): q = R^{-T} h - alpha u with
// the partial norms going to the beta array.
template <int CPW, bool WIDE>
__global__ void __launch_bounds__(BLK) k_trmv_t(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N,
                                                const double* __restrict__ t,
                                                const double* __restrict__ v,
                                                double* __restrict__ q,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ pnQ) {
  __shared__ double red[4];
  const Item it = items[blockIdx.x];
  const int j = it.j, p = it.p, i = j % N;
  const DevProb& pr = P[p];
  if (plan_stopped(pr)) return;
  const int64_t k = pr.k;
  const double* __restrict__ R = pr.Rinv + int64_t(sc[j].li) * k * k;
  const double* __restrict__ tv = t + pr.offS * N + int64_t(i) * k;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t cbase = int64_t(it.blk) * (4 * CPW) + wv * CPW;
  double acc[CPW];
#pragma unroll
  for (int q2 = 0; q2 < CPW; ++q2) acc[q2] = 0.0;
  const int64_t clast = min(k - 1, cbase + CPW - 1);
  for (int64_t r = lane; r <= clast; r += 64) {
    const double tr = tv[r];
#pragma unroll
    for (int q2 = 0; q2 < CPW; ++q2) {
      const int64_t c = cbase + q2;
      if (c < k && r <= c) acc[q2] = fma(R[r + c * k], tr, acc[q2]);
    }
  }
  const Scal& S = sc[j];
  double nrm = 0.0;
#pragma unroll
  for (int q2 = 0; q2 < CPW; ++q2) {
    const double s = warp_sum(acc[q2]);
    const int64_t c = cbase + q2;
    if (c < k) {
      const int64_t idx = (pr.offS + c) * N + i;
      const double nv = s - (WIDE ? S.alpha : S.beta_new) * v[idx];
      if (lane == 0) q[idx] = nv;
      nrm += nv * nv;
    }
  }
  if (lane != 0) nrm = 0.0;
  const double tot = block_sum(nrm, red);
  if (threadIdx.x == 0) pnQ[((WIDE ? pr.pnN : pr.pnQ) + it.blk) * N + i] = tot;
}

// ------------------------------------------------------------ fin_alpha ----
__global__ void __launch_bounds__(BLK) k_fin_alpha(const DevProb* __restrict__ P, int N,
                                                   const double* __restrict__ pnQ,
                                                   Scal* __restrict__ sc, int init, double tol,
                                                   int maxit) {
  __shared__ double red[4];
  const int j = blockIdx.x, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  if (plan_stopped(pr)) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < pr.nblkQ; b += BLK) v += pnQ[(pr.pnQ + b) * N + i];
  const double s = block_sum(v, red);
  if (threadIdx.x != 0) return;
  Scal& S = sc[j];
  const double alpha = sqrt(s);
  if (init) {
    S.alpha = alpha;
    S.rhobar = alpha;
    S.anorm2 = 0.0;
    S.iters = 0;
    S.upd = 0;
    S.cx = 0.0;
    S.ce = 0.0;
    if (!S.active) {
      S.ialpha = 0.0;
      S.ucoef = 0.0;
      return;
    }
    if (!isfinite(alpha)) {
      S.status = TIK_ST_NONFINITE;
      S.active = 0;
      S.tdone = int64_t(wall_clock64());
      S.ialpha = 0.0;
      S.ucoef = 0.0;
      return;
    }
    if (alpha == 0.0) {   // A^T b = 0: x = 0 is the solution
      S.status = TIK_ST_CONVERGED;
      S.active = 0;
      S.tdone = int64_t(wall_clock64());
      S.ialpha = 0.0;
      S.ucoef = 0.0;
      S.relres = 0.0;
      return;
    }
    S.ialpha = 1.0 / alpha;
    S.ucoef = alpha * S.ibeta;
    S.beta = S.beta_new;
    return;
  }
  if (!S.active) {
    S.upd = 0;
    S.ialpha = 0.0;
    S.ucoef = 0.0;
    return;
  }
  const double beta = S.beta_new;
  S.anorm2 += S.alpha * S.alpha + beta * beta;
  const double rho = hypot(S.rhobar, beta);
  const double cs = S.rhobar / rho, sn = beta / rho;
  const double theta = sn * alpha;
  const double rhobar = -cs * alpha;
  const double phi = cs * S.phibar;
  const double phibar = sn * S.phibar;
  const double tau = sn * phi;
  S.cx = phi / rho;
  S.ce = theta / rho;
  S.upd = 1;
  S.iters += 1;
  const double rnorm = phibar;
  const double arnorm = alpha * fabs(tau);
  const double anorm = sqrt(S.anorm2);
  const double test1 = rnorm / S.bnorm;
  const double test2 = (rnorm > 0.0) ? arnorm / (anorm * rnorm) : 0.0;
  S.rnorm = rnorm;
  S.arnorm = arnorm;
  S.relres = test2;
  if (!(isfinite(alpha) && isfinite(beta) && isfinite(rho) && rho > 0.0)) {
    S.status = TIK_ST_NONFINITE;
    S.active = 0;
    S.tdone = int64_t(wall_clock64());
    S.upd = 0;
    S.ialpha = 0.0;
    S.ucoef = 0.0;
    return;
  }
  if (test1 <= tol || test2 <= tol || alpha == 0.0) {
    S.status = TIK_ST_CONVERGED;
    S.active = 0;
    S.tdone = int64_t(wall_clock64());
  } else if (S.iters >= maxit) {
    S.status = TIK_ST_MAXIT;
    S.active = 0;
    S.tdone = int64_t(wall_clock64());
  }
  S.alpha = alpha;
  S.beta = beta;
  S.rhobar = rhobar;
  S.phibar = phibar;
  S.ialpha = alpha > 0.0 ? 1.0 / alpha : 0.0;
  S.ucoef = alpha * S.ibeta;
}

// ----------------------------------------------------------------- trmv ----
// w[r] = ialpha sum_{c >= r} Rinv[r, c] v~[c]; v = ialpha v~; x, e updates.
// 256 threads = 16 rows x 16 column slices; a wave reads 16 consecutive rows
// of 4 columns (full 128-byte lines) per load.
// WIDE: y = R^{-1} q / beta and u = q / beta (no x, e updates).
template <bool WIDE>
__global__ void __launch_bounds__(BLK) k_trmv(const DevProb* __restrict__ P,
                                              const Item* __restrict__ items, int N,
                                              const double* __restrict__ q,
                                              double* __restrict__ v, double* __restrict__ w,
                                              double* __restrict__ x, double* __restrict__ e,
                                              const Scal* __restrict__ sc, int init) {
  __shared__ double red[16][17];
  const Item it = items[blockIdx.x];
  const int j = it.j, p = it.p, i = j % N;
  const DevProb& pr = P[p];
  if (plan_stopped(pr)) return;
  const int64_t k = pr.k;
  const double* __restrict__ R = pr.Rinv + int64_t(sc[j].li) * k * k;
  const int tr = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int64_t r0 = int64_t(it.blk) * 16;
  const int64_t r = r0 + tr;
  const double* __restrict__ qv = q + pr.offS * N + i;   // q[(offS + c) * N + i] = qv[c * N]
  double acc = 0.0;
  if (r < k) {
    int64_t c = r0 + sl;
    for (; c + 48 < k; c += 64) {
      const double r_0 = R[r + c * k], r_1 = R[r + (c + 16) * k];
      const double r_2 = R[r + (c + 32) * k], r_3 = R[r + (c + 48) * k];
      acc = fma(r_0, qv[c * N], acc);
      acc = fma(r_1, qv[(c + 16) * N], acc);
      acc = fma(r_2, qv[(c + 32) * N], acc);
      acc = fma(r_3, qv[(c + 48) * N], acc);
    }
    for (; c < k; c += 16) acc = fma(R[r + c * k], qv[c * N], acc);
  }
  red[sl][tr] = acc;
  __syncthreads();
  if (sl != 0 || r >= k) return;
  double sum = 0.0;
#pragma unroll
  for (int q2 = 0; q2 < 16; ++q2) sum += red[q2][tr];
  const Scal& S = sc[j];
  const double scale = WIDE ? S.ibeta : S.ialpha;
  const double wr = sum * scale;
  const int64_t idx = (pr.offS + r) * N + i;
  v[idx] = q[idx] * scale;
  w[idx] = wr;
  if (WIDE) return;
  if (init) {
    x[idx] = 0.0;
    e[idx] = wr;
  } else if (S.upd) {
    const double eo = e[idx];
    x[idx] += S.cx * eo;
    e[idx] = wr - S.ce * eo;
  }
}

// --------------------------------------------------------- bookkeeping -----
__global__ void k_scal_init(Scal* sc, int J, int N, const double* __restrict__ lams,
                            const int32_t* __restrict__ pre_status,
                            const int32_t* __restrict__ lidx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  Scal S = {};
  S.li = lidx[j];
  S.lam = lams[j];
  S.sqlam = sqrt(S.lam);
  S.active = 1;
  S.status = TIK_ST_MAXIT;
  S.tstart = int64_t(wall_clock64());
  S.tdone = S.tstart;
  if (pre_status && pre_status[j] != TIK_ST_CONVERGED) {
    S.active = 0;
    S.status = pre_status[j];
  }
  sc[j] = S;
}

__global__ void k_count_active(const Scal* __restrict__ sc, int J, int32_t* out) {
  __shared__ int red[4];
  int c = 0;
  for (int j = threadIdx.x; j < J; j += BLK) c += sc[j].active;
  c = warp_sum(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// ===================================================== mixed precision (IR) ==
// Refinement of the augmented system [I A; A^T -lam I] [r; x] = [b; 0] in
// FP64 (Bjorck's iterative refinement for least squares, adapted to the
// Tikhonov term): with s = A x kept in FP64,
//   f = b - r - s,  g = A^T r - lam x        (FP64 residuals)
//   dx = argmin || [A; sqrt(lam) I] dx - [f; g / sqrt(lam)] ||   (inner LSQR)
//   x += dx,  s += A dx,  r += f - A dx.
// The inner solve runs with FP32 products (or FP64 for lambdas where FP32
// stops contracting); residuals, R^{-1} and x stay FP64.

__global__ void k_to_f32(const double* __restrict__ src, int64_t m, int64_t n, int64_t lda,
                         float* __restrict__ dst) {
  const int64_t total = m * n;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e % m, c = e / m;
    dst[e] = float(src[r + c * lda]);
  }
}

// f = b - r - s over all long rows of all problems (row-major, NF lambdas).
__global__ void k_ir_f(const DevProb* __restrict__ P, const Item* __restrict__ items, int rb,
                       int NF, const double* __restrict__ r, const double* __restrict__ s,
                       double* __restrict__ f, int first) {
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  for (int e = threadIdx.x; e < rb * NF; e += BLK) {
    const int64_t row = int64_t(it.blk) * rb + e / NF;
    const int i = e % NF;
    if (row >= pr.m) continue;
    const int64_t idx = (pr.offL + row) * NF + i;
    f[idx] = first ? pr.b[row] : pr.b[row] - r[idx] - s[idx];
  }
}

// Inner right-hand side [f; g / sqrt(lam)] gathered for the inner plan's
// lambda list, zero for lambdas not solved this sweep (use[j] == 0).
template <typename TC>
__global__ void __launch_bounds__(BLK) k_init_u_ir(const DevProb* __restrict__ P,
                                                   const Item* __restrict__ itN, int nItN, int rbN,
                                                   const Item* __restrict__ itB, int N, int NF,
                                                   int l0, const Scal* __restrict__ sc,
                                                   const int32_t* __restrict__ use,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ g,
                                                   TC* __restrict__ ut, double* __restrict__ ub,
                                                   double* __restrict__ pnN, double* __restrict__ pnB) {
  __shared__ double red[BLK];
  const bool top = int(blockIdx.x) < nItN;
  const Item it = top ? itN[blockIdx.x] : itB[blockIdx.x - nItN];
  const DevProb& pr = P[it.p];
  const int64_t rows = top ? pr.m : pr.n;
  const int64_t rb = top ? rbN : VB;
  const int64_t r0 = int64_t(it.blk) * rb;
  const int64_t r1 = min(rows, r0 + rb);
  double* pn = top ? pnN + (pr.pnN + it.blk) * N : pnB + (pr.pnB + it.blk) * N;
  const int rpp = BLK / N;                    // rows per pass, as in k_init_u
  const int t = threadIdx.x, i = t % N, rr = t / N;
  double loc = 0.0;
  if (rr < rpp) {
    const Scal& S = sc[it.p * N + i];
    const int li = S.li - l0;
    const bool on = use[it.p * N + i] != 0;
    const double isq = 1.0 / S.sqlam;
    for (int64_t r = r0 + rr; r < r1; r += rpp) {
      double v;
      if (top) {
        v = on ? f[(pr.irL + r) * NF + li] : 0.0;
        const TC vc = TC(v);
        ut[(pr.offL + r) * N + i] = vc;
        v = double(vc);
      } else {
        v = on ? g[(pr.irS + r) * NF + li] * isq : 0.0;
        ub[(pr.offS + r) * N + i] = v;
      }
      loc += v * v;
    }
  }
  red[t] = loc;
  __syncthreads();
  if (t < N) {
    double sum = 0.0;
    for (int j = 0; j < rpp; ++j) sum += red[t + j * N];
    pn[t] = sum;
  }
}

// dx[:, li] = inner x[:, i] where the inner solve of lambda li finished with a
// usable status.
__global__ void k_ir_scatter(const DevProb* __restrict__ P, int N, int NF, int l0,
                             const Scal* __restrict__ sc, const int32_t* __restrict__ use,
                             const double* __restrict__ xin, double* __restrict__ dx) {
  const int j = blockIdx.y, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  const Scal& S = sc[j];
  const bool ok = use[j] && (S.status == TIK_ST_CONVERGED || S.status == TIK_ST_MAXIT);
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < pr.n;
       c += int64_t(gridDim.x) * blockDim.x)
    if (ok) dx[(pr.irS + c) * NF + (S.li - l0)] = xin[(pr.offS + c) * N + i];
}

// x += dx; s += a; r += f - a.  Long rows for (r, s), short rows for x.
__global__ void k_ir_update_long(const DevProb* __restrict__ P, const Item* __restrict__ items,
                                 int rb, int NF, const double* __restrict__ f,
                                 const double* __restrict__ a, double* __restrict__ r,
                                 double* __restrict__ s) {
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  for (int e = threadIdx.x; e < rb * NF; e += BLK) {
    const int64_t row = int64_t(it.blk) * rb + e / NF;
    const int i = e % NF;
    if (row >= pr.m) continue;
    const int64_t idx = (pr.offL + row) * NF + i;
    const double av = a[idx];
    s[idx] += av;
    r[idx] += f[idx] - av;
  }
}

// x += dx and the per-(problem, lambda) squared norms of dx and of the new x.
__global__ void __launch_bounds__(BLK) k_ir_update_x(const DevProb* __restrict__ P, int NF,
                                                     const double* __restrict__ dx,
                                                     double* __restrict__ x,
                                                     double* __restrict__ nrm) {
  __shared__ double red[4];
  const int j = blockIdx.x, p = j / NF, i = j % NF;
  const DevProb& pr = P[p];
  double sd = 0.0, sx = 0.0;
  for (int64_t c = threadIdx.x; c < pr.n; c += BLK) {
    const int64_t idx = (pr.offS + c) * NF + i;
    const double d = dx[idx];
    const double nx = x[idx] + d;
    x[idx] = nx;
    sd += d * d;
    sx += nx * nx;
  }
  const double td = block_sum(sd, red);
  const double tx = block_sum(sx, red);
  if (threadIdx.x == 0) {
    nrm[2 * j] = td;
    nrm[2 * j + 1] = tx;
  }
}

// Copy the inner solves' iteration counts and statuses out per global lambda.
__global__ void k_ir_inner_stats(const DevProb* __restrict__ P, int J, int N, int NF, int l0,
                                 const Scal* __restrict__ sc, const int32_t* __restrict__ use,
                                 int32_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int p = j / N;
  const Scal& S = sc[j];
  const int g = P[p].gp * NF + (S.li - l0);
  out[2 * g] = use[j] ? S.iters : 0;
  out[2 * g + 1] = use[j] ? S.status : -1;
}

// Per-lambda outputs of a refined group, scattered from one table the host
// fills (one record per lambda the refinement wrote).
struct OutRec {
  int64_t gpos;
  int32_t it, st;
  double rel;
};

__global__ void k_scatter_outs(const OutRec* __restrict__ rec, int n, int32_t* __restrict__ iters,
                               int32_t* __restrict__ status, double* __restrict__ relres) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const OutRec r = rec[i];
  if (iters) iters[r.gpos] = r.it;
  if (status) status[r.gpos] = r.st;
  if (relres) relres[r.gpos] = r.rel;
}

__global__ void k_ir_write(const DevProb* __restrict__ P, int NF, const double* __restrict__ x,
                           const int32_t* __restrict__ ok, double* const* __restrict__ Xout,
                           int32_t l0) {
  const int j = blockIdx.y, p = j / NF, i = j % NF;
  const DevProb& pr = P[p];
  if (!ok[j]) return;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < pr.n;
       c += int64_t(gridDim.x) * blockDim.x)
    Xout[p][c + int64_t(l0 + i) * pr.n] = x[(pr.offS + c) * NF + i];
}

// ============================================================ wide problems ==
// Algorithm 2 (m < n): LSQR on M = R^{-T} [A sqrt(lam) I] from z = 0, so the
// minimum-norm z results and x is its top n entries (eq. regLLSunderiter).
//   beta u  = R^{-T} (A v_top + sqrt(lam) v_bot) - alpha u
//   alpha v = [A^T (R^{-1} u); sqrt(lam) R^{-1} u] - beta v
// "long" rows are the n columns of A (v_top, d_top, x), "short" rows the m rows
// (u, y = R^{-1} u, v_bot, d_bot, z_bot).  A v_top contracts over the long
// dimension: column chunks write partial products that k_wide_h sums.

// h (lambda-major) = sum_ch part + sqrt(lam) v_bot             (EPI 0)
// out[r, i]        = b[r] - sum_ch part - lam * yv[r, i]        (EPI 1, FP64 residual)
template <typename TC, int NC, int EPI>
__global__ void __launch_bounds__(BLK) k_wide_h(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N,
                                                const TC* __restrict__ part,
                                                const double* __restrict__ vb,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ out) {
  constexpr int RR = BLK / NC;
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t m = pr.m;
  const int64_t r = int64_t(it.blk) * RR + threadIdx.x / NC;
  const int i = threadIdx.x % NC;
  if (r >= m || i >= N) return;
  double s = 0.0;
  const TC* src = part + (pr.pnOff + r) * N + i;
#pragma unroll 8   // the chunk partials are independent loads: keep several in flight
  for (int ch = 0; ch < pr.nchN; ++ch) s += double(src[int64_t(ch) * m * N]);
  const Scal& S = sc[it.p * N + i];
  if (EPI == 0)
    out[pr.offS * N + int64_t(i) * m + r] = s + S.sqlam * vb[(pr.offS + r) * N + i];
  else
    out[(pr.offS + r) * N + i] = pr.b[r] - s - S.lam * vb[(pr.offS + r) * N + i];
}

// h = b (or the refinement right-hand side), lambda-major.
__global__ void k_wide_init_h(const DevProb* __restrict__ P, const Item* __restrict__ items,
                              int N, int NF, int l0, const Scal* __restrict__ sc,
                              const int32_t* __restrict__ use, const double* __restrict__ rhs,
                              double* __restrict__ t) {
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  for (int e = threadIdx.x; e < BLK * N; e += BLK) {
    const int64_t r = int64_t(it.blk) * BLK + e / N;
    const int i = e % N;
    if (r >= pr.m) continue;
    double v = pr.b[r];
    if (rhs) {
      const Scal& S = sc[it.p * N + i];
      v = use[it.p * N + i] ? rhs[(pr.irS + r) * NF + (S.li - l0)] : 0.0;
    }
    t[pr.offS * N + int64_t(i) * pr.m + r] = v;
  }
}

// v~ = [A^T y - beta v_top; sqrt(lam) y - beta v_bot] and its partial norms.
// One thread per (row, lambda): a block covers 256 / NC rows of all NC = 2^lgnc
// lambda slots, so consecutive threads touch consecutive entries of the
// row-major vectors.  Items: long blocks (blk < ceil(n / rows)), then short
// blocks over m; the partial squared norm of each block and lambda goes to pnQ.
template <typename TC>
__global__ void __launch_bounds__(BLK) k_wide_v(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N, int lgnc,
                                                const TC* __restrict__ part,
                                                const double* __restrict__ y,
                                                double* __restrict__ vt, double* __restrict__ vb,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ pnQ) {
  __shared__ double sh[BLK];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int RB = BLK >> lgnc;
  const int i = threadIdx.x & ((1 << lgnc) - 1);
  const int nL = int(cdiv(pr.n, RB));
  const bool lng = it.blk < nL;
  const int64_t r = int64_t(lng ? it.blk : it.blk - nL) * RB + (threadIdx.x >> lgnc);
  const int64_t rows = lng ? pr.n : pr.m;
  double v = 0.0;
  if (r < rows && i < N) {
    const Scal& S = sc[it.p * N + i];
    if (lng) {
      const int64_t idx = (pr.offL + r) * N + i;
      const double nv = double(part[(pr.ptOff + r) * N + i]) - S.beta_new * vt[idx];
      vt[idx] = nv;
      v = nv * nv;
    } else {
      const int64_t idx = (pr.offS + r) * N + i;
      const double nv = S.sqlam * y[idx] - S.beta_new * vb[idx];
      vb[idx] = nv;
      v = nv * nv;
    }
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  if (int(threadIdx.x) < N) {
    double tot = 0.0;
    for (int q = 0; q < RB; ++q) tot += sh[(q << lgnc) + threadIdx.x];
    pnQ[(pr.pnQ + it.blk) * N + threadIdx.x] = tot;
  }
}

// v = v~ / alpha; z += (phi/rho) d; d = v - (theta/rho) d (top: x, d_top;
// bottom: z_bot, d_bot).  Same (row, lambda) thread mapping as k_wide_v.
__global__ void __launch_bounds__(BLK) k_wide_upd(const DevProb* __restrict__ P,
                                                  const Item* __restrict__ items, int N, int lgnc,
                                                  double* __restrict__ vt, double* __restrict__ dt,
                                                  double* __restrict__ xt, double* __restrict__ vb,
                                                  double* __restrict__ db, double* __restrict__ zb,
                                                  const Scal* __restrict__ sc, int init) {
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int RB = BLK >> lgnc;
  const int i = threadIdx.x & ((1 << lgnc) - 1);
  const int nL = int(cdiv(pr.n, RB));
  const bool lng = it.blk < nL;
  const int64_t r = int64_t(lng ? it.blk : it.blk - nL) * RB + (threadIdx.x >> lgnc);
  const int64_t rows = lng ? pr.n : pr.m;
  if (r >= rows || i >= N) return;
  double* V = lng ? vt : vb;
  double* D = lng ? dt : db;
  double* Z = lng ? xt : zb;
  const Scal& S = sc[it.p * N + i];
  const int64_t idx = ((lng ? pr.offL : pr.offS) + r) * N + i;
  const double nv = V[idx] * S.ialpha;
  V[idx] = nv;
  if (init) {
    D[idx] = nv;
    Z[idx] = 0.0;
  } else if (S.upd) {
    const double d = D[idx];
    Z[idx] += S.cx * d;
    D[idx] = nv - S.ce * d;
  }
}

// X_p[:, li] = x (long rows) where the status allows.
__global__ void k_wide_write(const DevProb* __restrict__ P, int N, const double* __restrict__ x,
                             const Scal* __restrict__ sc, double* const* __restrict__ Xout,
                             const int32_t* __restrict__ jmap, int32_t* iters, int32_t* status,
                             double* relres) {
  const int j = blockIdx.y, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  const Scal& S = sc[j];
  const bool ok = S.status == TIK_ST_CONVERGED || S.status == TIK_ST_MAXIT;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < pr.n;
       c += int64_t(gridDim.x) * blockDim.x)
    if (ok && Xout[p]) Xout[p][c + int64_t(S.li) * pr.n] = x[(pr.offL + c) * N + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int g = jmap[j];
    if (iters) iters[g] = S.iters;
    if (status) status[g] = S.status;
    if (relres) relres[g] = S.relres;
  }
}

// ============================================================ host driver ===

void tile_autoload();

namespace {

// Item tables and partial-buffer sizes of the low-rank apply kernels.
struct LrTables {
  std::vector<Item> itLP, itLC, itLE, itLF;
  int64_t totLP = 0, totLC = 0, totLO = 0;
  void clear() {
    itLP.clear(); itLC.clear(); itLE.clear(); itLF.clear();
    totLP = totLC = totLO = 0;
  }
};

// Device copies of one LrTables.
struct LrDev {
  Item *itLP, *itLC, *itLE, *itLF;
  double *lpart, *lcoef, *lopart;
};

void take_lr(Arena& a, const LrTables& t, LrDev& d) {
  d.itLP = a.take<Item>(t.itLP.size());
  d.itLC = a.take<Item>(t.itLC.size());
  d.itLE = a.take<Item>(t.itLE.size());
  d.itLF = a.take<Item>(t.itLF.size());
  d.lpart = a.take<double>(size_t(t.totLP));
  d.lcoef = a.take<double>(size_t(t.totLC));
  d.lopart = a.take<double>(size_t(t.totLO));
}

LrItems lr_items(const LrTables& t, const LrDev& d) {
  return LrItems{d.itLP, d.itLC, d.itLE, d.itLF, int(t.itLP.size()), int(t.itLC.size()),
                 int(t.itLE.size()), int(t.itLF.size())};
}

LrBufs lr_bufs(const LrDev& d) { return LrBufs{d.lpart, d.lcoef, d.lopart}; }

// One set of (problem, lambda-range) solved together.
struct Plan {
  int N = 0, NC = 1, rbN = 64;
  std::vector<int> pidx;      // global problem index per local problem
  std::vector<int> lsel;      // lambda indices solved (the same list for every problem)
  std::vector<DevProb> P;
  std::vector<Item> itN, itB, itT, itQ, itR, itM;
  // A W tail (single-problem plans): row blocks tailBlk0.. are computed as
  // tailQ column pieces of tailPW columns (partial products of the rows from
  // tailBlk0 * 128 on, then summed and applied by k_gemm_n_tail_fin)
  int64_t tailBlk0 = 0, tailPW = 0, tailMt = 0;
  int tailQ = 0;
  int64_t tailNX = 0;                   // norm partials of the sum's sub-blocks 1.. (tailPn)
  DevProb Ptail = {};
  std::vector<Item> itTail;
  std::vector<Item> itNT;               // the row blocks before the tail, then its pieces (j = 1)
  LrTables lr;                          // low-rank apply: proj, expand, fin
  bool lowrank = false;
  int cpw = 16;
  int cbT = 64;        // columns per gemm_t block
  int64_t totL = 0, totS = 0, totPT = 0, nbN = 0, nbB = 0, nbQ = 0;
  int J = 0;
};

struct Bufs {
  DevProb* P;
  Item *itN, *itB, *itT, *itQ, *itR, *itM;
  DevProb* Ptail;     // the A W tail's problem (rows from the tail on)
  Item* itNT;         // one launch's items: the row blocks before the tail, then its pieces
  void* tailPart;     // the tail pieces' partial products (compute type)
  double* tailPn;     // norm partials of the tail sum's sub-blocks 1..
  LrDev lr;
  Scal* sc;
  void* ut;
  double *ub, *v, *q, *w, *e, *x, *t;
  float* w32;      // FP32 copy of w for the FP32 products A w
  void* part;
  double *pnN, *pnB, *pnQ;
  int32_t* cnt;
  double** Xp;
  double* lams;
  int32_t* pre;
  int32_t* jmap;
  int32_t* lidx;
};

int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

// Lambda slots per pass: N rounded up to a power of two; 5 to 8 lambdas use
// 16 slots so that the products run on the matrix cores (the passes are
// bound by the reads of A, which do not grow with the padding).
int pick_nc(int N) {
  int nc = 1;
  while (nc < N) nc <<= 1;
  return nc == 8 ? 16 : nc;
}

// Low-rank apply tables of one problem (k = its short dimension; V holds the
// right singular vectors of a tall problem's sketch, the left ones of a wide
// problem's).  Buffer sizes depend on s only, so any subset of the lambdas
// fits the same space.  Returns the number of fin blocks (norm partials).
int32_t lowrank_items(const tik_precond_s* pc, int p, int lp, const std::vector<int>& lsel, int NC,
                      LrTables& t, DevProb& d) {
  const int N = int(lsel.size());
  const int64_t k = d.k, s = pc->srank[p];
  int64_t smax = 0;
  for (int gi : lsel) smax = std::max<int64_t>(smax, pc->si[size_t(p) * pc->N + gi]);
  d.V = pc->V[p];
  d.S = pc->S[p];
  d.s = s;
  d.smax = smax;
  // columns per projection block: 128 on the matrix cores, 4 CPW otherwise
  const int cols = NC >= 16 ? 128 : 4 * (NC >= 32 ? 2 : 4);
  const int64_t cbs = std::max<int64_t>(1, cdiv(s, cols));
  int64_t nch = std::max<int64_t>(1, std::min<int64_t>(1024 / cbs, cdiv(k, 64)));
  const int64_t rch = cdiv(cdiv(k, nch), 64) * 64;
  nch = cdiv(k, rch);
  d.lrRch = rch;
  d.lrNch = int32_t(nch);
  d.lrNjc = int32_t(cdiv(smax, 256));
  d.lrPart = t.totLP;
  d.lrCoef = t.totLC;
  d.lrOpart = t.totLO;
  t.totLP += nch * s * N;
  t.totLC += s * N;
  t.totLO += cdiv(s, 256) * k * N;
  for (int64_t ch = 0; ch < nch; ++ch)
    for (int64_t jb = 0; jb < cdiv(smax, cols); ++jb) t.itLP.push_back({lp, int32_t(jb), int32_t(ch), 0});
  for (int64_t cb = 0; cb < cdiv(smax * N, 256); ++cb) t.itLC.push_back({lp, int32_t(cb), 0, 0});
  for (int64_t jc = 0; jc < d.lrNjc; ++jc)
    for (int64_t rb = 0; rb < cdiv(k, 256); ++rb) t.itLE.push_back({lp, int32_t(rb), int32_t(jc), 0});
  const int64_t nf = cdiv(k, 256 / NC);
  for (int64_t fb = 0; fb < nf; ++fb) t.itLF.push_back({lp, int32_t(fb), 0, 0});
  return int32_t(nf);
}

// ------------------------------------------------------------ tile table ----
// Launch shapes of the products over A per shape class: rows of A per gemm_n
// block (128 or 256; matrix-core tiles), columns per gemm_t block (64 or 128)
// and the number of product blocks the row or column split of a batch aims
// at.  A class is (orientation, FP32 storage, lambda slots per pass, log2 of
// the largest m and of the largest n, one / few / many problems).  Entries
// come from tik_tune (which times every candidate on the caller's problems)
// or from a table file (tik_tune_load; the file tuning.txt beside the library
// is read on first use); classes without an entry use the defaults below.
struct TileKey {
  int wide, a32, nc, lm, ln, lp;
  bool operator<(const TileKey& o) const {
    return std::tie(wide, a32, nc, lm, ln, lp) < std::tie(o.wide, o.a32, o.nc, o.lm, o.ln, o.lp);
  }
};
struct Tile {
  int rbN, cbT, blocks;
};
std::mutex g_tile_mu;
std::map<TileKey, Tile> g_tiles;
std::once_flag g_tile_once;
thread_local const Tile* t_tile_override = nullptr;   // set by the tuner
thread_local std::string t_last_tile;

int floor_log2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << (r + 1)) <= v) ++r;
  return r;
}

TileKey tile_key(int wide, const tik_problem* probs, const std::vector<int>& pidx, bool a32, int nc) {
  int64_t mm = 1, nn = 1;
  for (int k : pidx) {
    mm = std::max(mm, probs[k].m);
    nn = std::max(nn, probs[k].n);
  }
  const int np = int(pidx.size());
  return TileKey{wide, a32 ? 1 : 0, nc, floor_log2(mm), floor_log2(nn), np == 1 ? 0 : (np <= 16 ? 1 : 2)};
}

Tile tile_default(int wide) { return wide ? Tile{256, 128, 2048} : Tile{128, 64, 2048}; }

Tile tile_for(const TileKey& key, bool* tuned) {
  if (t_tile_override) {
    *tuned = true;
    return *t_tile_override;
  }
  tile_autoload();
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tiles.find(key);
  *tuned = it != g_tiles.end();
  return *tuned ? it->second : tile_default(key.wide);
}

void note_tile(const char* what, const TileKey& k, const Tile& t, bool tuned, int nc) {
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "%s lambda slots %d: gemm_n rows %d, gemm_t cols %d, product blocks %d (%s; class wide=%d "
                "a32=%d nc=%d lm=%d ln=%d lp=%d)",
                what, nc, t.rbN, t.cbT, t.blocks, tuned ? "tuned" : "default", k.wide, k.a32, k.nc, k.lm,
                k.ln, k.lp);
  t_last_tile = buf;
}

// The sum of the A W tail's column pieces (k_gemm_n_tail_fin): TAILF threads
// per block, TAILR rows per block, TAILS blocks per 128-row block of the tail.
static constexpr int TAILF = 512, TAILR = 16, TAILS = 128 / TAILR;

void make_plan(const tik_problem* probs, const tik_precond_s* pc, const std::vector<int>& pidx,
               const std::vector<int>& lsel, Plan& pl, const void* const* Aover = nullptr,
               const int64_t* ldover = nullptr) {
  const int N = int(lsel.size());
  pl.N = N;
  pl.NC = pick_nc(N);
  bool a32 = Aover != nullptr;
  for (int k : pidx) a32 |= probs[k].a_dtype == TIK_F32;
  const TileKey key = tile_key(0, probs, pidx, a32, pl.NC);
  bool tuned = false;
  const Tile tl = tile_for(key, &tuned);
  note_tile("tall", key, tl, tuned, pl.NC);
  // rows per gemm_n block and columns per gemm_t block: the table's on the
  // matrix cores, fixed for the few-lambda VALU kernels
  pl.rbN = pl.NC >= 16 ? tl.rbN : pl.NC >= 8 ? 256 : 64;
  pl.cpw = 4;          // columns per wave in R^{-T} t: low registers, high occupancy
  pl.cbT = pl.NC >= 16 ? tl.cbT : 64;
  pl.pidx = pidx;
  pl.lsel = lsel;
  pl.P.clear();
  pl.itN.clear(); pl.itB.clear(); pl.itT.clear(); pl.itQ.clear(); pl.itR.clear(); pl.itM.clear();
  pl.lr.clear();
  pl.totL = pl.totS = pl.totPT = pl.nbN = pl.nbB = pl.nbQ = 0;
  pl.lowrank = pc->route == TIK_ROUTE_LOWRANK;
  const int np = int(pidx.size());
  // gemm_t row chunks: one target length for the whole batch (about 2048
  // blocks, at most 8192 rows each), so the blocks of large and small problems
  // of a ragged batch are of similar length
  int64_t work = 0;
  for (int lp = 0; lp < np; ++lp) work += cdiv(probs[pidx[lp]].n, pl.cbT) * probs[pidx[lp]].m;
  const int64_t rtarget =
      std::min<int64_t>(8192, std::max<int64_t>(512, cdiv(cdiv(work, tl.blocks), 32) * 32));
  for (int lp = 0; lp < np; ++lp) {
    const tik_problem& g = probs[pidx[lp]];
    DevProb d = {};
    d.A = Aover ? Aover[pidx[lp]] : g.A;
    d.m = g.m;
    d.n = g.n;
    d.lda = ldover ? ldover[pidx[lp]] : g.lda;
    d.a_f32 = Aover ? 1 : (g.a_dtype == TIK_F32);
    d.wide = 0;
    d.b = g.b;
    d.offL = pl.totL;
    d.offS = pl.totS;
    d.offR = d.offL;
    d.offC = d.offS;
    d.irL = d.offL;
    d.irS = d.offS;
    d.gp = pidx[lp];
    d.cchunk = g.n;
    d.nchN = 1;
    d.pnOff = 0;
    d.k = g.n;
    if (pc->route == TIK_ROUTE_CHOL) d.Rinv = pc->Rinv[pidx[lp]];
    d.nblkN = int32_t(cdiv(g.m, pl.rbN));
    d.nblkB = int32_t(cdiv(g.n, VB));
    d.nblkQ = int32_t(cdiv(g.n, 4 * pl.cpw));
    if (pl.lowrank) d.nblkQ = lowrank_items(pc, pidx[lp], lp, lsel, pl.NC, pl.lr, d);
    d.pnN = pl.nbN;
    d.pnB = pl.nbB;
    d.pnQ = pl.nbQ;
    const int64_t cb = cdiv(g.n, pl.cbT);
    int64_t nch = cdiv(g.m, rtarget);
    const int64_t rch = cdiv(cdiv(g.m, nch), 32) * 32;
    nch = cdiv(g.m, rch);
    d.rchunk = rch;
    d.nchT = int32_t(nch);
    d.ptOff = pl.totPT;
    for (int b = 0; b < d.nblkN; ++b) pl.itN.push_back({lp, b, 0, 0});
    for (int b = 0; b < d.nblkB; ++b) pl.itB.push_back({lp, b, 0, 0});
    for (int64_t ch = 0; ch < nch; ++ch)
      for (int64_t c = 0; c < cb; ++c) pl.itT.push_back({lp, int32_t(c), int32_t(ch), 0});
    if (!pl.lowrank) {
      for (int i = 0; i < N; ++i)
        for (int b = 0; b < d.nblkQ; ++b) pl.itQ.push_back({lp, b, 0, lp * N + i});
      for (int i = 0; i < N; ++i)
        for (int64_t b = 0; b < cdiv(g.n, 16); ++b) pl.itM.push_back({lp, int32_t(b), 0, lp * N + i});
    }
    for (int64_t b = 0; b < cdiv(g.n, BLK / pl.NC); ++b) pl.itR.push_back({lp, int32_t(b), 0, 0});
    pl.totL += g.m;
    pl.totS += g.n;
    pl.totPT += nch * g.n;
    pl.nbN += d.nblkN;
    pl.nbB += d.nblkB;
    pl.nbQ += d.nblkQ;
    pl.P.push_back(d);
  }
  // The triangular products' blocks differ in length (block b of R^{-T} t reads
  // (b + 1) blocks of rows, row block b of R^{-1} q reads k - 16 b columns):
  // dispatch the longest first so the short ones fill the tail.
  auto q_work = [&](const Item& it) { return (int64_t(it.blk) + 1) * 4 * pl.cpw; };
  auto m_work = [&](const Item& it) { return pl.P[size_t(it.p)].k - 16 * int64_t(it.blk); };
  std::stable_sort(pl.itQ.begin(), pl.itQ.end(),
                   [&](const Item& a, const Item& b) { return q_work(a) > q_work(b); });
  std::stable_sort(pl.itM.begin(), pl.itM.end(),
                   [&](const Item& a, const Item& b) { return m_work(a) > m_work(b); });
  // product blocks of a ragged batch: the longest first (rows x columns of A)
  auto t_work = [&](const Item& it) {
    const DevProb& d = pl.P[size_t(it.p)];
    return std::min(d.rchunk, d.m - int64_t(it.ch) * d.rchunk);
  };
  if (np > 1) {
    std::stable_sort(pl.itT.begin(), pl.itT.end(),
                     [&](const Item& a, const Item& b) { return t_work(a) > t_work(b); });
    // k_gemm_t_mfma gives XCD x the item range [x per, (x + 1) per): deal the
    // sorted items round-robin over those ranges so every XCD gets a similar
    // mix, longest first
    const size_t nit = pl.itT.size(), per = (nit + 7) / 8;
    std::vector<Item> dealt(nit);
    std::vector<size_t> fill(8, 0);
    size_t x = 0;
    for (size_t i = 0; i < nit; ++i) {
      while (x * per + fill[x] >= std::min(nit, (x + 1) * per)) x = (x + 1) % 8;
      dealt[x * per + fill[x]++] = pl.itT[i];
      x = (x + 1) % 8;
    }
    pl.itT.swap(dealt);
  }
  std::stable_sort(pl.itN.begin(), pl.itN.end(), [&](const Item& a, const Item& b) {
    return pl.P[size_t(a.p)].n > pl.P[size_t(b.p)].n;
  });
  // The A W launch of B row blocks with C resident at a time ends with a round
  // of B mod C blocks, each bound by one CU's matrix-core rate for its whole
  // row block (200000 x 2000, 32 lambdas: 1563 blocks, 768 resident, 0.79 ms
  // per launch against 0.70 ms for 1536 blocks).  When that round is at most
  // half full, its row blocks are computed instead as column pieces spread
  // over the whole GPU: the pieces follow the other row blocks in the same
  // launch (they fill the compute units as the last full round drains) and
  // store their partial products, and k_gemm_n_tail_fin sums them in piece
  // order and applies the update (the kernel boundary orders the two, so no
  // fences).
  pl.tailQ = 0;
  pl.tailNX = 0;
  pl.itTail.clear();
  pl.itNT.clear();
  pl.tailBlk0 = pl.P.empty() ? 0 : pl.P[0].nblkN;
  if (option_gemm_n_tail() && np == 1 && pl.NC >= 16 && N <= TAILF / TAILR && pl.rbN == 128 &&
      pl.P[0].n >= 256) {
    const DevProb& d = pl.P[0];
    const int64_t B = d.nblkN, C = gemm_n_resident(d.a_f32, 0, pl.NC);
    const int64_t r = C > 0 ? B % C : 0;
    if (C > 0 && B > C && r > 0 && 2 * r <= C) {
      int64_t q = std::min<int64_t>(std::min<int64_t>(64, C / r), d.n / 64);
      const int64_t pw = cdiv(cdiv(d.n, q), 16) * 16;
      q = cdiv(d.n, pw);
      if (q >= 2) {
        pl.tailQ = int(q);
        pl.tailPW = pw;
        pl.tailBlk0 = B - r;
        const int64_t row0 = pl.tailBlk0 * 128;
        pl.tailMt = d.m - row0;
        DevProb t = d;
        t.A = static_cast<const char*>(d.A) + row0 * (d.a_f32 ? 4 : 8);
        t.m = pl.tailMt;
        t.cchunk = pw;
        t.nchN = int32_t(q);
        t.pnOff = 0;
        pl.Ptail = t;
        for (int64_t b = 0; b < r; ++b)
          for (int64_t c = 0; c < q; ++c) pl.itTail.push_back({0, int32_t(b), int32_t(c), 0});
        pl.tailNX = r * (TAILS - 1);
        pl.itNT.assign(pl.itN.begin(), pl.itN.begin() + pl.tailBlk0);
        for (Item t2 : pl.itTail) {
          t2.j = 1;
          pl.itNT.push_back(t2);
        }
      }
    }
  }
  pl.J = np * N;
}

// Sum of the tail's column-piece products in piece order, then the EPI 0
// update u~ = A W - ucoef u~ of those rows and their squared-norm partials
// (single-problem plans).  Block g takes rows TAILR (g mod TAILS) .. of 128-row
// block g / TAILS of the tail: spread over about TAILS times as many compute
// units as 128-row blocks would be, since one unit's share of the pieces is
// bound by its own bandwidth.  Thread t handles lambda t % N of row t / N
// (N <= TAILF / TAILR, so one row each); its pieces are loaded eight at a time
// and added in piece order.  Sub-block 0 of each 128-row block writes that
// block's norm-partial slot, the others the extra partials pnX that k_fin_beta
// adds (every sub-block writes its partial, zero where it has no rows).
template <typename TC>
__global__ void __launch_bounds__(TAILF) k_gemm_n_tail_fin(const DevProb* __restrict__ P, int N,
                                                           int64_t blk0, int64_t mt, int q,
                                                           const TC* __restrict__ part,
                                                           TC* __restrict__ ut,
                                                           const Scal* __restrict__ sc,
                                                           double* __restrict__ pnN,
                                                           double* __restrict__ pnX) {
  __shared__ double red[TAILF];
  const DevProb& pr = P[0];
  if (plan_stopped(pr)) return;
  const int t = threadIdx.x, i = t % N, rr = t / N;
  const int64_t blk = blockIdx.x / TAILS;
  const int sub = int(blockIdx.x % TAILS);
  const int64_t r = blk * 128 + int64_t(sub) * TAILR + rr;
  double loc = 0.0;
  if (rr < TAILR && r < mt) {
    const TC* pp = part + r * N + i;
    const int64_t stride = mt * N;
    TC acc = TC(0);
    int c = 0;
    for (; c + 8 <= q; c += 8) {
      TC v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[int64_t(c + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; c < q; ++c) acc += pp[int64_t(c) * stride];
    const int64_t idx = (pr.offR + blk0 * 128 + r) * N + i;
    const TC nv = TC(acc - TC(sc[i].ucoef) * ut[idx]);
    ut[idx] = nv;
    loc = double(nv) * double(nv);
  }
  red[t] = loc;
  __syncthreads();
  if (t < N) {
    double s = 0.0;
    for (int j = 0; j < TAILR; ++j) s += red[t + j * N];
    if (sub == 0) pnN[(pr.pnN + blk0 + blk) * N + t] = s;
    else pnX[(blk * (TAILS - 1) + sub - 1) * N + t] = s;
  }
}


void take_bufs(Arena& a, const Plan& pl, size_t tc, Bufs& b) {
  const int N = pl.N;
  b.P = a.take<DevProb>(pl.P.size());
  b.itN = a.take<Item>(pl.itN.size());
  b.itB = a.take<Item>(pl.itB.size());
  b.itT = a.take<Item>(pl.itT.size());
  b.itQ = a.take<Item>(pl.itQ.size());
  b.itR = a.take<Item>(pl.itR.size());
  b.itM = a.take<Item>(pl.itM.size());
  b.Ptail = a.take<DevProb>(pl.tailQ ? 1 : 0);
  b.itNT = a.take<Item>(pl.itNT.size());
  b.tailPart = a.take<double>(size_t(pl.tailQ) * size_t(pl.tailMt) * size_t(N));
  b.tailPn = a.take<double>(size_t(pl.tailNX) * size_t(N));
  take_lr(a, pl.lr, b.lr);
  b.sc = a.take<Scal>(pl.J);
  b.ut = a.take<char>(size_t(pl.totL) * N * tc);
  b.ub = a.take<double>(size_t(pl.totS) * N);
  b.v = a.take<double>(size_t(pl.totS) * N);
  b.q = a.take<double>(size_t(pl.totS) * N);
  b.w = a.take<double>(size_t(pl.totS) * N);
  b.w32 = a.take<float>(size_t(pl.totS) * N);
  b.e = a.take<double>(size_t(pl.totS) * N);
  b.x = a.take<double>(size_t(pl.totS) * N);
  b.t = a.take<double>(size_t(pl.totS) * N);
  b.part = a.take<char>(size_t(pl.totPT) * N * tc);
  b.pnN = a.take<double>(size_t(pl.nbN) * N);
  b.pnB = a.take<double>(size_t(pl.nbB) * N);
  b.pnQ = a.take<double>(size_t(pl.nbQ) * N);
  b.cnt = a.take<int32_t>(1);
  b.Xp = a.take<double*>(pl.P.size());
  b.lams = a.take<double>(pl.J);
  b.pre = a.take<int32_t>(pl.J);
  b.jmap = a.take<int32_t>(pl.J);
  b.lidx = a.take<int32_t>(pl.J);
}

// FP64 -> FP32 copy of count values.
__global__ void k_vec_to_f32(const double* __restrict__ x, int64_t count, float* __restrict__ y) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += int64_t(gridDim.x) * blockDim.x)
    y[e] = float(x[e]);
}

// FP32 copy of an FP64 vector block for the FP32 products (read by every block
// of the product: converted once instead of in every block).
static int vec_to_f32(const double* x, int64_t count, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_vec_to_f32, dim3(unsigned(std::min<int64_t>(cdiv(count, 256), 1024))), dim3(256),
                     0, st, x, count, y);
  TIK_LAUNCHED("k_vec_to_f32");
  return TIK_OK;
}

template <typename TA, typename TC, int NC>
struct Kern {
  static int gemm_n(const Plan& pl, const Bufs& b, hipStream_t st) {
    ProfScope ps("gemm_n", st);
    if (NC >= 16) {
      constexpr bool c32 = std::is_same<TC, float>::value;
      if (c32) TIK_TRY(vec_to_f32(b.w, int64_t(pl.totS) * pl.N, b.w32, st));
      const void* W = c32 ? static_cast<const void*>(b.w32) : static_cast<const void*>(b.w);
      constexpr int a32 = std::is_same<TA, float>::value;
      if (!pl.tailQ)
        return launch_gemm_n_mfma(a32, c32, NC, 0, pl.rbN, b.P, b.itN, int(pl.itN.size()), pl.N, W,
                                  b.ut, nullptr, b.sc, b.pnN, st);
      TIK_TRY(launch_gemm_n_mfma(a32, c32, NC, 3, pl.rbN, b.P, b.itNT, int(pl.itNT.size()), pl.N, W,
                                 b.ut, nullptr, b.sc, b.pnN, st, b.Ptail, b.tailPart));
      hipLaunchKernelGGL(k_gemm_n_tail_fin<TC>,
                         dim3(unsigned((int64_t(pl.itN.size()) - pl.tailBlk0) * TAILS)), dim3(TAILF), 0,
                         st, b.P, pl.N, pl.tailBlk0, pl.tailMt, pl.tailQ,
                         static_cast<const TC*>(b.tailPart), static_cast<TC*>(b.ut), b.sc, b.pnN,
                         b.tailPn);
      TIK_LAUNCHED("k_gemm_n_tail_fin");
      return TIK_OK;
    }
    if (NC >= 8)
      hipLaunchKernelGGL((k_gemm_n<TA, TC, NC, 256, 1, 0>), dim3(unsigned(pl.itN.size())), dim3(BLK),
                         0, st, b.P, b.itN, pl.N, b.w, static_cast<TC*>(b.ut), nullptr, b.sc, b.pnN);
    else
      hipLaunchKernelGGL((k_gemm_n<TA, TC, NC, 64, 4, 0>), dim3(unsigned(pl.itN.size())), dim3(BLK),
                         0, st, b.P, b.itN, pl.N, b.w, static_cast<TC*>(b.ut), nullptr, b.sc, b.pnN);
    TIK_LAUNCHED("k_gemm_n");
    return TIK_OK;
  }
  static int gemm_t(const Plan& pl, const Bufs& b, hipStream_t st) {
    ProfScope ps("gemm_t", st);
    if (NC >= 16)
      return launch_gemm_t_mfma(std::is_same<TA, float>::value, std::is_same<TC, float>::value, 0, NC,
                                pl.cbT, b.P, b.itT, int(pl.itT.size()), pl.N, b.ut, b.part, st);
    hipLaunchKernelGGL((k_gemm_t<TA, TC, TC, NC>), dim3(unsigned(pl.itT.size())), dim3(BLK), 0, st,
                       b.P, b.itT, pl.N, static_cast<const TC*>(b.ut), int64_t(pl.N),
                       static_cast<TC*>(b.part));
    TIK_LAUNCHED("k_gemm_t");
    return TIK_OK;
  }
};

template <typename TC>
int vec_steps_u(const Plan& pl, const Bufs& b, hipStream_t st, bool init, const double* rhs_top,
                const double* rhs_bot) {
  ProfScope ps("vec", st);
  if (init) {
    hipLaunchKernelGGL(k_init_u<TC>, dim3(unsigned(pl.itN.size() + pl.itB.size())), dim3(BLK), 0,
                       st, b.P, b.itN, int(pl.itN.size()), pl.rbN, b.itB, pl.N, rhs_top, rhs_bot,
                       static_cast<TC*>(b.ut), b.ub, b.pnN, b.pnB);
    TIK_LAUNCHED("k_init_u");
  } else {
    hipLaunchKernelGGL(k_vec_bot, dim3(unsigned(pl.itB.size())), dim3(BLK), 0, st, b.P, b.itB, pl.N,
                       b.w, b.ub, b.sc, b.pnB);
    TIK_LAUNCHED("k_vec_bot");
  }
  hipLaunchKernelGGL(k_fin_beta, dim3(unsigned(pl.J)), dim3(BLK), 0, st, b.P, pl.N, b.pnN, b.pnB,
                     b.sc, init ? 1 : 0, static_cast<const double*>(b.tailPn), int(pl.tailNX));
  TIK_LAUNCHED("k_fin_beta");
  return TIK_OK;
}

template <typename TC, int NC>
int vec_steps_v(const Plan& pl, const Bufs& b, hipStream_t st, bool init, double tol, int maxit) {
  {
    ProfScope ps("vec", st);
    hipLaunchKernelGGL((k_reduce_t<TC, 0, NC>), dim3(unsigned(pl.itR.size())), dim3(BLK), 0, st, b.P,
                       b.itR, pl.N, static_cast<const TC*>(b.part), b.ub, b.sc, b.t);
    TIK_LAUNCHED("k_reduce_t");
  }
  if (pl.lowrank) {
    ProfScope ps("lr_apply", st);
    TIK_TRY(launch_lr_apply(pl.NC, 0, 1, b.P, lr_items(pl.lr, b.lr), pl.N, b.t, lr_bufs(b.lr),
                            b.q, b.v, b.w, b.x, b.e, b.sc, b.pnQ, init ? 1 : 0, st));
  } else {
    ProfScope ps("trmv_t", st);
    if (pl.cpw == 16)
      hipLaunchKernelGGL((k_trmv_t<16, false>), dim3(unsigned(pl.itQ.size())), dim3(BLK), 0, st, b.P,
                         b.itQ, pl.N, b.t, b.v, b.q, b.sc, b.pnQ);
    else
      hipLaunchKernelGGL((k_trmv_t<4, false>), dim3(unsigned(pl.itQ.size())), dim3(BLK), 0, st, b.P,
                         b.itQ, pl.N, b.t, b.v, b.q, b.sc, b.pnQ);
    TIK_LAUNCHED("k_trmv_t");
  }
  {
    ProfScope ps("vec", st);
    hipLaunchKernelGGL(k_fin_alpha, dim3(unsigned(pl.J)), dim3(BLK), 0, st, b.P, pl.N, b.pnQ, b.sc,
                       init ? 1 : 0, tol, maxit);
    TIK_LAUNCHED("k_fin_alpha");
  }
  if (pl.lowrank) {
    ProfScope ps("lr_apply", st);
    TIK_TRY(launch_lr_apply(pl.NC, 1, 1, b.P, lr_items(pl.lr, b.lr), pl.N, b.q, lr_bufs(b.lr),
                            b.q, b.v, b.w, b.x, b.e, b.sc, b.pnQ, init ? 1 : 0, st));
  } else {
    ProfScope ps("trmv", st);
    hipLaunchKernelGGL(k_trmv<false>, dim3(unsigned(pl.itM.size())), dim3(BLK), 0, st, b.P, b.itM,
                       pl.N, b.q, b.v, b.w, b.x, b.e, b.sc, init ? 1 : 0);
    TIK_LAUNCHED("k_trmv");
  }
  return TIK_OK;
}

int upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return TIK_OK;
  TIK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  return TIK_OK;
}

// Run LSQR to completion for one plan; x is left in b.x.
struct IrRhs {
  const int32_t* use;   // per solve of the plan: solved this sweep
  const double* f;      // long rows x NF
  const double* g;      // short rows x NF
  int NF;
  int l0;               // global index of refinement column 0
};

// ------------------------------------------------------ iteration control --
// The solve loops queue LSQR iterations ahead of the host: every iteration
// ends with a one-block kernel that writes the number of still-active solves
// into the plan's live word, and every kernel of a later iteration returns at
// once when that word reads 0 (plan_stopped), leaving all state unchanged.
// The host looks at the count one step late: after queuing step c it waits for
// the count copied after step c - 1 (an async copy into one of two pinned host
// words per call, an event each), so the GPU always has work queued.
//
// A step is a chunk of T iterations captured once per call into a HIP graph
// and replayed (T from tik_set_option("graph_chunk"), default 4): a solve of
// I iterations makes ceil(I / T) + 1 host waits and replays at most two
// chunks past convergence, whose kernels return at once.  With T = 0, or
// while per-launch profiling is on, a step is one iteration launched directly.
std::mutex g_pin_mu;
std::vector<int32_t*> g_pin_free;   // pinned pairs, kept for the process

struct IterGate {
  int32_t* h = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool clean = false;               // no copy in flight: the pair may be reused
  int open() {
    {
      std::lock_guard<std::mutex> lk(g_pin_mu);
      if (!g_pin_free.empty()) {
        h = g_pin_free.back();
        g_pin_free.pop_back();
      }
    }
    if (!h) {
      void* p = nullptr;
      TIK_HIP(hipHostMalloc(&p, 2 * sizeof(int32_t), hipHostMallocDefault));
      h = static_cast<int32_t*>(p);
    }
    for (auto& e : ev) TIK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return TIK_OK;
  }
  // after step c is queued: copy the live count to host word c & 1, mark it
  int post(int c, const int32_t* cnt, hipStream_t st) {
    TIK_HIP(hipMemcpyAsync(h + (c & 1), cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TIK_HIP(hipEventRecord(ev[c & 1], st));
    return TIK_OK;
  }
  // wait for the count posted after step c; *zero: every solve has stopped
  int seen(int c, bool* zero) {
    TIK_HIP(hipEventSynchronize(ev[c & 1]));
    *zero = h[c & 1] == 0;
    return TIK_OK;
  }
  // products run again outside the loop (refinement residuals, later calls)
  int close(int32_t* cnt, hipStream_t st) {
    TIK_HIP(hipMemsetAsync(cnt, 1, sizeof(int32_t), st));
    for (auto& e : ev)
      if (e) TIK_HIP(hipEventSynchronize(e));
    clean = true;
    return TIK_OK;
  }
  ~IterGate() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h && clean) {
      std::lock_guard<std::mutex> lk(g_pin_mu);
      g_pin_free.push_back(h);
    }
  }
};

// Capture happens on a library stream of the calling thread (a capture records
// launches without running them); the graph is then replayed on the caller's
// stream, which may be the null stream where capture itself is not allowed.
int capture_stream(hipStream_t* out) {
  thread_local std::vector<hipStream_t> streams;
  int dev = 0;
  TIK_HIP(hipGetDevice(&dev));
  if (size_t(dev) >= streams.size()) streams.resize(size_t(dev) + 1, nullptr);
  if (!streams[size_t(dev)])
    TIK_HIP(hipStreamCreateWithFlags(&streams[size_t(dev)], hipStreamNonBlocking));
  *out = streams[size_t(dev)];
  return TIK_OK;
}

struct ChunkGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  ~ChunkGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
  }
  template <typename F>
  int capture(F& one, int T) {
    hipStream_t cs = nullptr;
    TIK_TRY(capture_stream(&cs));
    TIK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = TIK_OK;
    for (int t = 0; t < T && rc == TIK_OK; ++t) rc = one(cs);
    const hipError_t e = hipStreamEndCapture(cs, &g);   // always end, even after a failure
    TIK_TRY(rc);
    if (e != hipSuccess) {
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return TIK_EHIP;
    }
    TIK_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    return TIK_OK;
  }
};

// Queue iterations until every solve of the plan has stopped or maxit
// iterations are queued; `body(s)` queues one iteration's kernels on s.
template <typename Body>
int iterate(Body&& body, const Scal* sc, int J, int32_t* cnt, int maxit, hipStream_t st) {
  auto one = [&](hipStream_t s) -> int {
    TIK_TRY(body(s));
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(BLK), 0, s, sc, J, cnt);
    TIK_LAUNCHED("k_count_active");
    return TIK_OK;
  };
  if (noalloc_active()) {
    // nothing allocated: each count is read back into a host local after a
    // stream synchronization
    for (int it = 0; it < maxit; ++it) {
      TIK_TRY(one(st));
      int32_t h = 1;
      TIK_HIP(hipMemcpyAsync(&h, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      TIK_HIP(hipStreamSynchronize(st));
      if (h == 0) break;
    }
    TIK_HIP(hipMemsetAsync(cnt, 1, sizeof(int32_t), st));
    return TIK_OK;
  }
  IterGate gate;
  TIK_TRY(gate.open());
  const int T = std::min(maxit, option_chunk());
  if (T > 0 && !prof_active()) {
    ChunkGraph cg;
    TIK_TRY(cg.capture(one, T));
    int queued = 0;
    for (int c = 0; queued < maxit; ++c) {
      TIK_HIP(hipGraphLaunch(cg.exec, st));
      queued += T;
      TIK_TRY(gate.post(c, cnt, st));
      bool zero = false;
      if (c > 0) TIK_TRY(gate.seen(c - 1, &zero));
      if (zero) break;
    }
  } else {
    for (int it = 0; it < maxit; ++it) {
      TIK_TRY(one(st));
      TIK_TRY(gate.post(it, cnt, st));
      bool zero = false;
      if (it > 0) TIK_TRY(gate.seen(it - 1, &zero));
      if (zero) {   // the products of iteration `it` returned at once
        prof_drop_last("gemm_n");
        prof_drop_last("gemm_t");
        break;
      }
    }
  }
  return gate.close(cnt, st);
}

template <typename TA, typename TC, int NC>
int run_core(const Plan& pl, const Bufs& b, double tol, int maxit, hipStream_t st,
             const IrRhs* ir) {
  using K = Kern<TA, TC, NC>;
  hipLaunchKernelGGL(k_scal_init, dim3(unsigned(cdiv(pl.J, 256))), dim3(256), 0, st, b.sc, pl.J,
                     pl.N, b.lams, b.pre, b.lidx);
  TIK_LAUNCHED("k_scal_init");
  TIK_HIP(hipMemsetAsync(b.v, 0, size_t(pl.totS) * pl.N * sizeof(double), st));
  if (ir) {
    ProfScope ps("vec", st);
    hipLaunchKernelGGL(k_init_u_ir<TC>, dim3(unsigned(pl.itN.size() + pl.itB.size())), dim3(BLK), 0,
                       st, b.P, b.itN, int(pl.itN.size()), pl.rbN, b.itB, pl.N, ir->NF, ir->l0, b.sc, ir->use,
                       ir->f, ir->g, static_cast<TC*>(b.ut), b.ub, b.pnN, b.pnB);
    TIK_LAUNCHED("k_init_u_ir");
    hipLaunchKernelGGL(k_fin_beta, dim3(unsigned(pl.J)), dim3(BLK), 0, st, b.P, pl.N, b.pnN, b.pnB,
                       b.sc, 1, static_cast<const double*>(nullptr), 0);
    TIK_LAUNCHED("k_fin_beta");
  } else {
    TIK_TRY(vec_steps_u<TC>(pl, b, st, true, nullptr, nullptr));
  }
  TIK_TRY(K::gemm_t(pl, b, st));
  TIK_TRY((vec_steps_v<TC, NC>(pl, b, st, true, tol, maxit)));
  auto body = [&](hipStream_t s) -> int {
    TIK_TRY(K::gemm_n(pl, b, s));
    TIK_TRY(vec_steps_u<TC>(pl, b, s, false, nullptr, nullptr));
    TIK_TRY(K::gemm_t(pl, b, s));
    return vec_steps_v<TC, NC>(pl, b, s, false, tol, maxit);
  };
  return iterate(body, b.sc, pl.J, b.cnt, maxit, st);
}

template <typename TA, typename TC>
int run_core_nc(const Plan& pl, const Bufs& b, double tol, int maxit, hipStream_t st,
                const IrRhs* ir) {
  switch (pl.NC) {
    case 1: return run_core<TA, TC, 1>(pl, b, tol, maxit, st, ir);
    case 2: return run_core<TA, TC, 2>(pl, b, tol, maxit, st, ir);
    case 4: return run_core<TA, TC, 4>(pl, b, tol, maxit, st, ir);
    case 8: return run_core<TA, TC, 8>(pl, b, tol, maxit, st, ir);
    case 16: return run_core<TA, TC, 16>(pl, b, tol, maxit, st, ir);
    case 32: return run_core<TA, TC, 32>(pl, b, tol, maxit, st, ir);
  }
  set_error("internal: lambda batch wider than 32");
  return TIK_ENOTSUP;
}

// Upload a plan's tables and per-solve data.  Host staging vectors are kept
// in `keep` until the caller synchronizes.
int upload_plan(const Plan& pl, const Bufs& b, const tik_precond_s* pc, double* const* X,
                std::vector<std::vector<char>>& keep, hipStream_t st) {
  auto stash = [&](const void* src, size_t bytes) -> const void* {
    keep.emplace_back(static_cast<const char*>(src), static_cast<const char*>(src) + bytes);
    return keep.back().data();
  };
  std::vector<DevProb> P = pl.P;
  for (auto& d : P) d.live = b.cnt;
  TIK_HIP(hipMemsetAsync(b.cnt, 1, sizeof(int32_t), st));
  TIK_TRY(upload(b.P, stash(P.data(), P.size() * sizeof(DevProb)), P.size() * sizeof(DevProb), st));
  TIK_TRY(upload(b.itN, stash(pl.itN.data(), pl.itN.size() * sizeof(Item)), pl.itN.size() * sizeof(Item), st));
  TIK_TRY(upload(b.itB, stash(pl.itB.data(), pl.itB.size() * sizeof(Item)), pl.itB.size() * sizeof(Item), st));
  TIK_TRY(upload(b.itT, stash(pl.itT.data(), pl.itT.size() * sizeof(Item)), pl.itT.size() * sizeof(Item), st));
  TIK_TRY(upload(b.itQ, stash(pl.itQ.data(), pl.itQ.size() * sizeof(Item)), pl.itQ.size() * sizeof(Item), st));
  TIK_TRY(upload(b.itR, stash(pl.itR.data(), pl.itR.size() * sizeof(Item)), pl.itR.size() * sizeof(Item), st));
  TIK_TRY(upload(b.itM, stash(pl.itM.data(), pl.itM.size() * sizeof(Item)), pl.itM.size() * sizeof(Item), st));
  if (pl.tailQ) {
    DevProb t = pl.Ptail;
    t.live = b.cnt;
    TIK_TRY(upload(b.Ptail, stash(&t, sizeof(DevProb)), sizeof(DevProb), st));
    TIK_TRY(upload(b.itNT, stash(pl.itNT.data(), pl.itNT.size() * sizeof(Item)),
                   pl.itNT.size() * sizeof(Item), st));
  }
  const LrTables& lr = pl.lr;
  TIK_TRY(upload(b.lr.itLP, stash(lr.itLP.data(), lr.itLP.size() * sizeof(Item)), lr.itLP.size() * sizeof(Item), st));
  TIK_TRY(upload(b.lr.itLC, stash(lr.itLC.data(), lr.itLC.size() * sizeof(Item)), lr.itLC.size() * sizeof(Item), st));
  TIK_TRY(upload(b.lr.itLE, stash(lr.itLE.data(), lr.itLE.size() * sizeof(Item)), lr.itLE.size() * sizeof(Item), st));
  TIK_TRY(upload(b.lr.itLF, stash(lr.itLF.data(), lr.itLF.size() * sizeof(Item)), lr.itLF.size() * sizeof(Item), st));
  std::vector<double> lams(pl.J);
  std::vector<int32_t> pre(pl.J), jmap(pl.J), lidx(pl.J);
  std::vector<double*> xp(pl.P.size());
  for (size_t lp = 0; lp < pl.P.size(); ++lp) {
    const int p = pl.pidx[lp];
    for (int i = 0; i < pl.N; ++i) {
      const int gi = pl.lsel[i];
      lams[lp * pl.N + i] = pc->lams[size_t(p) * pc->N + gi];
      pre[lp * pl.N + i] = pc->status[size_t(p) * pc->N + gi];
      jmap[lp * pl.N + i] = p * pc->N + gi;
      lidx[lp * pl.N + i] = gi;
    }
    xp[lp] = X ? X[p] : nullptr;
  }
  TIK_TRY(upload(b.lidx, stash(lidx.data(), lidx.size() * 4), lidx.size() * 4, st));
  TIK_TRY(upload(b.lams, stash(lams.data(), lams.size() * 8), lams.size() * 8, st));
  TIK_TRY(upload(b.pre, stash(pre.data(), pre.size() * 4), pre.size() * 4, st));
  TIK_TRY(upload(b.jmap, stash(jmap.data(), jmap.size() * 4), jmap.size() * 4, st));
  TIK_TRY(upload(b.Xp, stash(xp.data(), xp.size() * sizeof(double*)), xp.size() * sizeof(double*), st));
  return TIK_OK;
}

__global__ void k_write_out_map(const DevProb* __restrict__ P, int N, const double* __restrict__ x,
                                const Scal* __restrict__ sc, double* const* __restrict__ Xout,
                                const int32_t* __restrict__ jmap, int32_t* iters, int32_t* status,
                                double* relres) {
  const int j = blockIdx.y;
  const int p = j / N, i = j % N;
  const DevProb& pr = P[p];
  const Scal& S = sc[j];
  const bool ok = S.status == TIK_ST_CONVERGED || S.status == TIK_ST_MAXIT;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < pr.n;
       c += int64_t(gridDim.x) * blockDim.x)
    if (ok && Xout[p]) Xout[p][c + int64_t(S.li) * pr.n] = x[(pr.offS + c) * N + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int g = jmap[j];
    if (iters) iters[g] = S.iters;
    if (status) status[g] = S.status;
    if (relres) relres[g] = S.relres;
  }
}

void groups_for(const tik_precond_s* pc, int32_t nprob, int32_t mode,
                std::vector<std::vector<int>>& gp, std::vector<std::vector<int>>& gl) {
  gp.clear(); gl.clear();
  const int N = pc->N;
  if (mode == TIK_PLAIN_F64_PER_LAMBDA) {
    for (int p = 0; p < nprob; ++p)
      for (int i = 0; i < N; ++i) {
        gp.push_back({p});
        gl.push_back({i});
      }
    return;
  }
  // batched: all problems, lambdas in groups of at most 32
  std::vector<int> ps;
  for (int p = 0; p < nprob; ++p) ps.push_back(p);
  for (int i0 = 0; i0 < N; i0 += 32) {
    std::vector<int> ls;
    for (int i = i0; i < std::min(N, i0 + 32); ++i) ls.push_back(i);
    gp.push_back(ps);
    gl.push_back(ls);
  }
}

// ------------------------------------------------------------ mixed driver --
struct MixedWs {
  std::vector<float*> A32;        // FP32 copies of FP64-stored problems (null if stored FP32)
  double *r, *s, *f, *a, *x, *dx, *g, *nrm;
  int32_t *use32, *use64, *stats, *ok;
  OutRec* rec;                    // per-lambda output records
  char* base32 = nullptr;         // inner FP32 plan region
  char* base64 = nullptr;         // inner FP64 plan region
  size_t cap32 = 0, cap64 = 0;
  char* baseF = nullptr;          // FP64 refinement plan region
  size_t capF = 0;
  bool converted = false;         // FP32 copies made
};

void all_lambdas(int N0, int N, std::vector<int>& ls) {
  ls.clear();
  for (int i = N0; i < N0 + N; ++i) ls.push_back(i);
}

// Lambda counts whose plans bound the workspace of every subset of NF lambdas:
// a plan's buffers grow with the count within one tile width (pick_nc), so the
// largest count of each width class (capped at NF) suffices.
std::vector<int> subset_sizes(int NF) {
  std::vector<int> out;
  for (int ng = 1; ng <= NF; ++ng)
    if (ng == NF || pick_nc(ng + 1) != pick_nc(ng)) out.push_back(ng);
  return out;
}

// Workspace layout of the mixed mode for lambda groups of at most 32.
// One copy of the records and one scatter instead of three small copies per lambda.
int scatter_outs(const std::vector<OutRec>& recs, OutRec* dev, int32_t* iters, int32_t* status,
                 double* relres, std::vector<std::vector<char>>& keep, hipStream_t st) {
  if (recs.empty() || (!iters && !status && !relres)) return TIK_OK;
  const char* h = reinterpret_cast<const char*>(recs.data());
  keep.emplace_back(h, h + recs.size() * sizeof(OutRec));
  TIK_HIP(hipMemcpyAsync(dev, keep.back().data(), recs.size() * sizeof(OutRec), hipMemcpyHostToDevice, st));
  const int n = int(recs.size());
  hipLaunchKernelGGL(k_scatter_outs, dim3(unsigned(cdiv(n, 256))), dim3(256), 0, st, dev, n, iters, status,
                     relres);
  TIK_LAUNCHED("k_scatter_outs");
  return TIK_OK;
}

size_t mixed_layout(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, Arena& a,
                    MixedWs& w) {
  std::vector<int> ps;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  const int NF = std::min(32, pc->N);
  std::vector<int> ls;
  all_lambdas(0, NF, ls);
  Plan pl;
  make_plan(p, pc, ps, ls, pl);
  w.A32.assign(size_t(nprob), nullptr);
  for (int k = 0; k < nprob; ++k)
    if (p[k].a_dtype == TIK_F64) w.A32[k] = a.take<float>(size_t(p[k].m) * size_t(p[k].n));
  const size_t L = size_t(pl.totL) * NF, S = size_t(pl.totS) * NF;
  w.r = a.take<double>(L);
  w.s = a.take<double>(L);
  w.f = a.take<double>(L);
  w.a = a.take<double>(L);
  w.x = a.take<double>(S);
  w.dx = a.take<double>(S);
  w.g = a.take<double>(S);
  w.nrm = a.take<double>(2 * size_t(pl.J));
  w.use32 = a.take<int32_t>(pl.J);
  w.use64 = a.take<int32_t>(pl.J);
  w.stats = a.take<int32_t>(2 * size_t(pl.J));
  w.ok = a.take<int32_t>(pl.J);
  w.rec = a.take<OutRec>(pl.J);
  std::vector<Plan> subs;                 // inner plans solve subsets of the lambdas
  for (int ng : subset_sizes(NF)) {
    std::vector<int> sub;
    all_lambdas(0, ng, sub);
    subs.emplace_back();
    make_plan(p, pc, ps, sub, subs.back());
  }
  auto region = [&](size_t tc, char*& base, size_t& cap) {
    cap = 0;
    for (const Plan& q : subs) {
      Arena m;
      Bufs b;
      take_bufs(m, q, tc, b);
      cap = std::max(cap, m.used + 256);
    }
    base = a.take<char>(cap);
  };
  region(sizeof(float), w.base32, w.cap32);
  region(sizeof(double), w.base64, w.cap64);
  region(sizeof(double), w.baseF, w.capF);
  return a.used;
}

template <typename TA>
int ir_products_t(const Plan& pf, const Bufs& bf, const double* U, hipStream_t st) {
  ProfScope ps("residual", st);
  if (pf.NC >= 16)
    return launch_gemm_t_mfma(std::is_same<TA, float>::value, 0, 1, pf.NC, pf.cbT, bf.P, bf.itT,
                              int(pf.itT.size()), pf.N, U, bf.part, st);
  switch (pf.NC) {
#define GT(nc) case nc: hipLaunchKernelGGL((k_gemm_t<TA, double, double, nc>), dim3(unsigned(pf.itT.size())), dim3(BLK), 0, st, bf.P, bf.itT, pf.N, U, int64_t(pf.N), static_cast<double*>(bf.part)); break;
    GT(1) GT(2) GT(4) GT(8)
#undef GT
  }
  TIK_LAUNCHED("k_gemm_t (refinement)");
  return TIK_OK;
}

template <typename TA>
int ir_products_n(const Plan& pf, const Bufs& bf, const double* W, double* out, hipStream_t st) {
  ProfScope ps("residual", st);
  if (pf.NC >= 16)
    return launch_gemm_n_mfma(std::is_same<TA, float>::value, 0, pf.NC, 1, pf.rbN, bf.P, bf.itN,
                              int(pf.itN.size()), pf.N, W, nullptr, out, bf.sc, nullptr, st);
  switch (pf.NC) {
#define GN(nc) case nc: hipLaunchKernelGGL((k_gemm_n<TA, double, nc, (nc >= 8 ? 256 : 64), (nc >= 8 ? 1 : 4), 1>), dim3(unsigned(pf.itN.size())), dim3(BLK), 0, st, bf.P, bf.itN, pf.N, W, static_cast<double*>(nullptr), out, bf.sc, static_cast<double*>(nullptr)); break;
    GN(1) GN(2) GN(4) GN(8)
#undef GN
  }
  TIK_LAUNCHED("k_gemm_n (refinement)");
  return TIK_OK;
}

template <int NC>
int ir_reduce_g(const Plan& pf, const Bufs& bf, const double* x, double* g, hipStream_t st) {
  hipLaunchKernelGGL((k_reduce_t<double, 1, NC>), dim3(unsigned(pf.itR.size())), dim3(BLK), 0, st,
                     bf.P, bf.itR, pf.N, static_cast<const double*>(bf.part), x, bf.sc, g);
  TIK_LAUNCHED("k_reduce_t (refinement)");
  return TIK_OK;
}

int ir_reduce_g_nc(const Plan& pf, const Bufs& bf, const double* x, double* g, hipStream_t st) {
  ProfScope ps("residual", st);
  switch (pf.NC) {
    case 1: return ir_reduce_g<1>(pf, bf, x, g, st);
    case 2: return ir_reduce_g<2>(pf, bf, x, g, st);
    case 4: return ir_reduce_g<4>(pf, bf, x, g, st);
    case 8: return ir_reduce_g<8>(pf, bf, x, g, st);
    case 16: return ir_reduce_g<16>(pf, bf, x, g, st);
    case 32: return ir_reduce_g<32>(pf, bf, x, g, st);
  }
  set_error("internal: refinement batch wider than 32");
  return TIK_ENOTSUP;
}

// One inner solve over the lambdas `sel` (global indices) with FP32 (f32 = true)
// or FP64 products; the result is scattered into w.dx.
template <typename TA64>
int inner_solve(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, const MixedWs& w,
                const Plan& pf, const std::vector<int>& sel, const std::vector<uint8_t>& use_h,
                int NF, int l0, bool f32, double tol, int maxit, hipStream_t st,
                std::vector<std::vector<char>>& keep) {
  // only the problems with a lambda to correct: a pass over A costs the same
  // for one lambda as for all of a problem's, so late sweeps, where few
  // lambdas are left, read only their problems
  std::vector<int> ps;
  for (int k = 0; k < nprob; ++k) {
    bool any = false;
    for (int li : sel) any |= use_h[size_t(k) * NF + size_t(li - l0)] != 0;
    if (any) ps.push_back(k);
  }
  if (ps.empty() || pf.P.size() != size_t(nprob)) {
    set_error("internal: inner solve without problems");
    return TIK_EINVAL;
  }
  std::vector<const void*> Aov(static_cast<size_t>(nprob));
  std::vector<int64_t> ldo(static_cast<size_t>(nprob));
  bool any_override = false;
  for (int k = 0; k < nprob; ++k) {
    const bool ov = f32 && w.A32[k];
    Aov[k] = ov ? static_cast<const void*>(w.A32[k]) : p[k].A;
    ldo[k] = ov ? p[k].m : p[k].lda;                 // the FP32 copy is packed
    any_override |= ov;
  }
  Plan pl;
  make_plan(p, pc, ps, sel, pl, any_override ? Aov.data() : nullptr,
            any_override ? ldo.data() : nullptr);
  {
    // the region is sized for all problems; a subset chunks its rows finer
    // and may need more partial rows: then take them all
    Arena m;
    Bufs mb;
    take_bufs(m, pl, f32 ? sizeof(float) : sizeof(double), mb);
    if (m.used > (f32 ? w.cap32 : w.cap64) && ps.size() < size_t(nprob)) {
      ps.clear();
      for (int k = 0; k < nprob; ++k) ps.push_back(k);
      make_plan(p, pc, ps, sel, pl, any_override ? Aov.data() : nullptr,
                any_override ? ldo.data() : nullptr);
    }
  }
  for (size_t lp = 0; lp < pl.P.size(); ++lp) {
    if (f32) pl.P[lp].a_f32 = 1;
    pl.P[lp].irL = pf.P[size_t(ps[lp])].offL;
    pl.P[lp].irS = pf.P[size_t(ps[lp])].offS;
  }
  Arena a;
  a.base = f32 ? w.base32 : w.base64;
  a.cap = f32 ? w.cap32 : w.cap64;
  Bufs b;
  take_bufs(a, pl, f32 ? sizeof(float) : sizeof(double), b);
  if (!a.fits()) {
    set_error("internal: inner plan exceeds its region");
    return TIK_EWORKSPACE;
  }
  TIK_TRY(upload_plan(pl, b, pc, nullptr, keep, st));
  std::vector<int32_t> use(size_t(pl.J));
  for (size_t lp = 0; lp < ps.size(); ++lp)
    for (size_t i = 0; i < sel.size(); ++i)
      use[lp * sel.size() + i] = use_h[size_t(ps[lp]) * NF + size_t(sel[i] - l0)];
  keep.emplace_back(reinterpret_cast<const char*>(use.data()),
                    reinterpret_cast<const char*>(use.data()) + use.size() * 4);
  int32_t* dUse = f32 ? w.use32 : w.use64;
  TIK_HIP(hipMemcpyAsync(dUse, keep.back().data(), use.size() * 4, hipMemcpyHostToDevice, st));
  IrRhs ir{dUse, w.f, w.g, NF, l0};
  // the inner plan's solves map to refinement columns sel[i] - l0: shift li
  // by l0 inside the scatter through the Scal lambda index
  if (f32)
    TIK_TRY((run_core_nc<float, float>(pl, b, tol, maxit, st, &ir)));
  else
    TIK_TRY((run_core_nc<TA64, double>(pl, b, tol, maxit, st, &ir)));
  int64_t maxn = 0;
  for (auto& d : pl.P) maxn = std::max(maxn, d.n);
  (void)l0;
  hipLaunchKernelGGL(k_ir_scatter, dim3(unsigned(cdiv(maxn, 256)), unsigned(pl.J)), dim3(256), 0,
                     st, b.P, pl.N, NF, l0, b.sc, dUse, b.x, w.dx);
  TIK_LAUNCHED("k_ir_scatter");
  hipLaunchKernelGGL(k_ir_inner_stats, dim3(unsigned(cdiv(pl.J, 256))), dim3(256), 0, st, b.P,
                     pl.J, pl.N, NF, l0, b.sc, dUse, w.stats);
  TIK_LAUNCHED("k_ir_inner_stats");
  return TIK_OK;
}

template <typename TA64>
int mixed_group(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, MixedWs& w,
                int l0, int NF, double tol, int maxit, double* const* X, int32_t* iters,
                int32_t* status, double* relres, hipStream_t st) {
  std::vector<int> ps;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  std::vector<int> lsel;
  all_lambdas(l0, NF, lsel);
  Plan pf;
  make_plan(p, pc, ps, lsel, pf);
  Arena af;
  af.base = w.baseF;
  af.cap = w.capF;
  Bufs bf;
  take_bufs(af, pf, sizeof(double), bf);
  if (!af.fits()) {
    set_error("internal: refinement plan exceeds its region");
    return TIK_EWORKSPACE;
  }
  std::vector<std::vector<char>> keep;
  TIK_TRY(upload_plan(pf, bf, pc, nullptr, keep, st));
  hipLaunchKernelGGL(k_scal_init, dim3(unsigned(cdiv(pf.J, 256))), dim3(256), 0, st, bf.sc, pf.J,
                     pf.N, bf.lams, bf.pre, bf.lidx);
  TIK_LAUNCHED("k_scal_init");
  const size_t L = size_t(pf.totL) * NF, S = size_t(pf.totS) * NF;
  TIK_HIP(hipMemsetAsync(w.r, 0, L * 8, st));
  TIK_HIP(hipMemsetAsync(w.s, 0, L * 8, st));
  TIK_HIP(hipMemsetAsync(w.x, 0, S * 8, st));
  const int J = pf.J;
  // host-side refinement state per (problem, lambda of the group)
  std::vector<int32_t> st_h(J, -1), it_h(J, 0);
  std::vector<double> dxrel(J, 1.0), rho(J, 1.0), rel_h(J, 0.0);
  std::vector<uint8_t> done(J, 0), want64(J, 0), was64(J, 0);
  for (int j = 0; j < J; ++j) {
    const int k = j / NF, i = j % NF;
    const int32_t pre = pc->status[size_t(k) * pc->N + l0 + i];
    if (pre != TIK_ST_CONVERGED) {
      st_h[j] = pre;
      done[j] = 1;
    }
  }
  // Lambdas where FP32 products cannot drive the refinement: its contraction
  // per sweep is about c * kappa(B) * u_32 (c ~ 12 measured), with kappa(B)^2
  // <= (||C|| + lambda) / lambda.  Such a lambda needs FP64 passes over A, and
  // a pass over A costs the same for one lambda as for all of them, so once
  // one lambda of the group needs FP64 the whole group is solved by batched
  // FP64 LSQR (refinement sweeps would only add passes).
  std::vector<int> hard;
  bool any_hard = false;
  for (int i = 0; i < NF; ++i)
    for (int k = 0; k < nprob; ++k) {
      const double lam = pc->lams[size_t(k) * pc->N + l0 + i];
      const double kap = std::sqrt((pc->cnorm[k] + lam) / lam);
      any_hard |= 12.0 * kap * std::ldexp(1.0, -24) > 0.25;
    }
  if (any_hard)
    for (int i = 0; i < NF; ++i) hard.push_back(l0 + i);
  if (!hard.empty()) {
    Plan ph;
    make_plan(p, pc, ps, hard, ph);
    Arena ah;
    ah.base = w.base64;
    ah.cap = w.cap64;
    Bufs bh;
    take_bufs(ah, ph, sizeof(double), bh);
    if (!ah.fits()) {
      set_error("internal: FP64 plan exceeds its region");
      return TIK_EWORKSPACE;
    }
    TIK_TRY(upload_plan(ph, bh, pc, X, keep, st));
    const double tol_h = std::max(1e-3 * tol, 1e-14);
    note_split(0, int32_t(hard.size()) * nprob);
    TIK_TRY((run_core_nc<TA64, double>(ph, bh, tol_h, maxit, st, nullptr)));
    int64_t mn = 0;
    for (auto& d : ph.P) mn = std::max(mn, d.n);
    hipLaunchKernelGGL(k_write_out_map, dim3(unsigned(cdiv(mn, 256)), unsigned(ph.J)), dim3(256), 0,
                       st, bh.P, ph.N, bh.x, bh.sc, bh.Xp, bh.jmap, iters, status, relres);
    TIK_LAUNCHED("k_write_out");
    TIK_HIP(hipStreamSynchronize(st));
    for (int li : hard)
      for (int k = 0; k < nprob; ++k) {
        const int j = k * NF + (li - l0);
        done[j] = 2;     // finished outside the refinement
      }
  }
  const int maxsweep = 12;
  const double tol32 = std::max(tol, 1e-6);
  {
    int32_t n32 = 0;
    for (int j = 0; j < J; ++j) n32 += done[j] == 0;
    note_split(n32, 0);
    if (n32 > 0 && !w.converted) {
      // FP32 copies of FP64-stored problems, made once per call
      ProfScope ps("residual", st);
      for (int k = 0; k < nprob; ++k)
        if (w.A32[k]) {
          const int64_t tot = p[k].m * p[k].n;
          hipLaunchKernelGGL(k_to_f32, dim3(unsigned(std::min<int64_t>(cdiv(tot, 256), 65536))),
                             dim3(256), 0, st, static_cast<const double*>(p[k].A), p[k].m, p[k].n,
                             p[k].lda, w.A32[k]);
          TIK_LAUNCHED("k_to_f32");
        }
      w.converted = true;
    }
  }
  std::vector<double> nrm(2 * size_t(J));
  std::vector<int32_t> stats(2 * size_t(J));
  for (int sweep = 1; sweep <= maxsweep; ++sweep) {
    bool any = false;
    for (int j = 0; j < J; ++j) any |= !done[j];
    if (!any) break;
    {
      ProfScope ps("residual", st);
      hipLaunchKernelGGL(k_ir_f, dim3(unsigned(pf.itN.size())), dim3(BLK), 0, st, bf.P, bf.itN,
                         pf.rbN, NF, w.r, w.s, w.f, sweep == 1 ? 1 : 0);
    }
    TIK_LAUNCHED("k_ir_f");
    if (sweep == 1) {
      TIK_HIP(hipMemsetAsync(w.g, 0, S * 8, st));
    } else {
      TIK_TRY(ir_products_t<TA64>(pf, bf, w.r, st));
      TIK_TRY(ir_reduce_g_nc(pf, bf, w.x, w.g, st));
    }
    // choose the inner precision per lambda (uniform across problems)
    std::vector<int> sel32, sel64;
    std::vector<uint8_t> use32(J, 0), use64(J, 0);
    for (int i = 0; i < NF; ++i) {
      bool act = false, hard = false;
      for (int k = 0; k < nprob; ++k) {
        const int j = k * NF + i;
        if (!done[j]) {
          act = true;
          hard |= want64[j] != 0;
        }
      }
      if (!act) continue;
      (hard ? sel64 : sel32).push_back(l0 + i);
      for (int k = 0; k < nprob; ++k) {
        const int j = k * NF + i;
        if (!done[j]) (hard ? use64 : use32)[j] = 1;
      }
    }
    double err64 = 1.0;
    for (int j = 0; j < J; ++j)
      if (use64[j]) err64 = std::min(err64, std::max(dxrel[j] * std::min(1.0, rho[j]), 1e-300));
    const double tol64 = std::min(1e-6, std::max(1e-14, 1e-3 * tol / std::max(err64, 1e-300)));
    TIK_HIP(hipMemsetAsync(w.dx, 0, S * 8, st));
    TIK_HIP(hipMemsetAsync(w.stats, 0xFF, 2 * size_t(J) * 4, st));
    if (!sel32.empty())
      TIK_TRY(inner_solve<TA64>(p, nprob, pc, w, pf, sel32, use32, NF, l0, true, tol32, maxit, st,
                                keep));
    if (!sel64.empty())
      TIK_TRY(inner_solve<TA64>(p, nprob, pc, w, pf, sel64, use64, NF, l0, false, tol64, maxit, st,
                                keep));
    TIK_TRY(ir_products_n<TA64>(pf, bf, w.dx, w.a, st));
    {
      ProfScope ps("residual", st);
      hipLaunchKernelGGL(k_ir_update_long, dim3(unsigned(pf.itN.size())), dim3(BLK), 0, st, bf.P,
                         bf.itN, pf.rbN, NF, w.f, w.a, w.r, w.s);
      hipLaunchKernelGGL(k_ir_update_x, dim3(unsigned(J)), dim3(BLK), 0, st, bf.P, NF, w.dx, w.x, w.nrm);
    }
    TIK_LAUNCHED("k_ir_update");
    TIK_HIP(hipMemcpyAsync(nrm.data(), w.nrm, nrm.size() * 8, hipMemcpyDeviceToHost, st));
    TIK_HIP(hipMemcpyAsync(stats.data(), w.stats, stats.size() * 4, hipMemcpyDeviceToHost, st));
    TIK_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < J; ++j) {
      if (done[j] || !(use32[j] || use64[j])) continue;
      it_h[j] += std::max(0, stats[2 * j]);
      const int32_t ist = stats[2 * j + 1];
      if (ist == TIK_ST_NOTPD || ist == TIK_ST_NONFINITE) {
        st_h[j] = ist;
        done[j] = 1;
        continue;
      }
      const double nx = std::sqrt(nrm[2 * j + 1]), nd = std::sqrt(nrm[2 * j]);
      if (!std::isfinite(nx) || !std::isfinite(nd)) {
        st_h[j] = TIK_ST_NONFINITE;
        done[j] = 1;
        continue;
      }
      const double rel = nx > 0.0 ? nd / nx : 0.0;
      const double r_k = sweep == 1 ? 1.0 : rel / std::max(dxrel[j], 1e-300);
      rel_h[j] = rel;
      // converged: the correction itself is below tol, or the sweeps contract
      // (r_k < 0.1) and the error left after this correction, about r_k rel,
      // is a hundred times below tol.  r_k is a contraction only from the third
      // sweep on (the first correction is the whole solution).
      if (rel <= tol || (sweep >= 3 && r_k < 0.1 && r_k * rel <= 1e-2 * tol)) {
        st_h[j] = TIK_ST_CONVERGED;
        done[j] = 1;
      } else if (use64[j] && r_k > 0.9 && sweep > 2) {
        st_h[j] = TIK_ST_IR_STALL;
        done[j] = 1;
      } else if (sweep == maxsweep) {
        st_h[j] = TIK_ST_MAXIT;
        done[j] = 1;
      }
      // next inner precision: FP64 where FP32 contraction is poor, FP32 right
      // after an FP64 sweep (the FP32 sweep then confirms the correction)
      const bool poor = (sweep == 2 && rel > 5e-5) || (sweep >= 3 && r_k > 0.15);
      want64[j] = use64[j] ? 0 : (poor ? 1 : 0);
      was64[j] = use64[j];
      rho[j] = sweep == 1 ? 1.0 : r_k;
      dxrel[j] = rel;
    }
  }
  for (int j = 0; j < J; ++j)
    if (!done[j]) st_h[j] = TIK_ST_MAXIT;
  // outputs (lambdas solved by the FP64 batch were written already)
  std::vector<int32_t> okv(J);
  for (int j = 0; j < J; ++j)
    okv[j] = done[j] != 2 && (st_h[j] == TIK_ST_CONVERGED || st_h[j] == TIK_ST_MAXIT ||
                              st_h[j] == TIK_ST_IR_STALL) ? 1 : 0;
  std::vector<double*> xp(static_cast<size_t>(nprob));
  for (int k = 0; k < nprob; ++k) xp[k] = X[k];
  keep.emplace_back(reinterpret_cast<const char*>(okv.data()), reinterpret_cast<const char*>(okv.data()) + J * 4);
  TIK_HIP(hipMemcpyAsync(w.ok, keep.back().data(), size_t(J) * 4, hipMemcpyHostToDevice, st));
  keep.emplace_back(reinterpret_cast<const char*>(xp.data()),
                    reinterpret_cast<const char*>(xp.data()) + xp.size() * sizeof(double*));
  TIK_HIP(hipMemcpyAsync(bf.Xp, keep.back().data(), xp.size() * sizeof(double*), hipMemcpyHostToDevice, st));
  int64_t maxn = 0;
  for (auto& d : pf.P) maxn = std::max(maxn, d.n);
  hipLaunchKernelGGL(k_ir_write, dim3(unsigned(cdiv(maxn, 256)), unsigned(J)), dim3(256), 0, st,
                     bf.P, NF, w.x, w.ok, bf.Xp, l0);
  TIK_LAUNCHED("k_ir_write");
  // per-lambda outputs at global positions k * N + l0 + i (refined lambdas only)
  std::vector<OutRec> recs;
  for (int j = 0; j < J; ++j)
    if (done[j] != 2)
      recs.push_back(OutRec{int64_t(j / NF) * pc->N + l0 + (j % NF), it_h[j], st_h[j], rel_h[j]});
  TIK_TRY(scatter_outs(recs, w.rec, iters, status, relres, keep, st));
  TIK_HIP(hipStreamSynchronize(st));
  return TIK_OK;
}

int mixed_run(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, double tol,
              int32_t maxit, double* const* X, int32_t* iters, int32_t* status, double* relres,
              void* dws, size_t dws_bytes, hipStream_t st) {
  Arena a;
  a.base = static_cast<char*>(dws);
  a.cap = dws_bytes;
  MixedWs w;
  mixed_layout(p, nprob, pc, a, w);
  if (!a.fits()) {
    set_error("tik_lsqr_batch: workspace too small");
    return TIK_EWORKSPACE;
  }
  const bool f32 = p[0].a_dtype == TIK_F32;
  for (int l0 = 0; l0 < pc->N; l0 += 32) {
    const int NF = std::min(32, pc->N - l0);
    if (f32)
      TIK_TRY(mixed_group<float>(p, nprob, pc, w, l0, NF, tol, maxit, X, iters, status, relres, st));
    else
      TIK_TRY(mixed_group<double>(p, nprob, pc, w, l0, NF, tol, maxit, X, iters, status, relres, st));
  }
  return TIK_OK;
}

// ------------------------------------------------------------- wide driver --
struct WPlan {
  int N = 0, NC = 1, rbN = 64, cpw = 4, cbT = 64;
  std::vector<int> pidx, lsel;
  std::vector<DevProb> P;
  std::vector<Item> itNs, itT, itQ, itM, itR, itV, itH;
  LrTables lr;
  bool lowrank = false;
  int64_t totL = 0, totS = 0, totPN = 0, totPT = 0, nbN = 0, nbQ = 0;
  int J = 0;
};

struct WBufs {
  DevProb* P;
  Item *itNs, *itT, *itQ, *itM, *itR, *itV, *itH;
  LrDev lr;
  Scal* sc;
  void *partN, *partT;
  double *vt, *dt, *xt, *u, *q, *y, *vb, *db, *zb, *t, *pnN, *pnQ;
  float* y32;      // FP32 copy of y for the FP32 products A^T y
  float* w32;      // FP32 copy of the n-side vector for the FP32 products A w
  int32_t* cnt;
  double** Xp;
  double* lams;
  int32_t *pre, *jmap, *lidx;
};

void make_plan_wide(const tik_problem* probs, const tik_precond_s* pc, const std::vector<int>& pidx,
                    const std::vector<int>& lsel, WPlan& pl, const void* const* Aover = nullptr,
                    const int64_t* ldover = nullptr) {
  const int N = int(lsel.size());
  pl = WPlan();
  pl.N = N;
  pl.NC = pick_nc(N);
  bool a32 = Aover != nullptr;
  for (int k : pidx) a32 |= probs[k].a_dtype == TIK_F32;
  const TileKey key = tile_key(1, probs, pidx, a32, pl.NC);
  bool tuned = false;
  const Tile tl = tile_for(key, &tuned);
  note_tile("wide", key, tl, tuned, pl.NC);
  // rows per gemm_n block (v_top is re-read per block) and columns per gemm_t
  // block (y is re-read per block): the table's on the matrix cores
  pl.rbN = pl.NC >= 16 ? tl.rbN : pl.NC >= 8 ? 256 : 64;
  pl.cpw = 4;          // columns per wave in R^{-T} t: low registers, high occupancy
  pl.cbT = pl.NC >= 16 ? tl.cbT : 64;
  pl.pidx = pidx;
  pl.lsel = lsel;
  pl.lowrank = pc->route == TIK_ROUTE_LOWRANK;
  const int np = int(pidx.size());
  int64_t rowblocks = 0;
  for (int lp = 0; lp < np; ++lp) rowblocks += cdiv(probs[pidx[lp]].m, pl.rbN);
  for (int lp = 0; lp < np; ++lp) {
    const tik_problem& g = probs[pidx[lp]];
    DevProb d = {};
    d.A = Aover ? Aover[pidx[lp]] : g.A;
    d.m = g.m;
    d.n = g.n;
    d.lda = ldover ? ldover[pidx[lp]] : g.lda;
    d.a_f32 = Aover ? 1 : (g.a_dtype == TIK_F32);
    d.wide = 1;
    d.b = g.b;
    d.offL = pl.totL;
    d.offS = pl.totS;
    d.offR = d.offS;
    d.offC = d.offL;
    d.irL = d.offL;
    d.irS = d.offS;
    d.gp = pidx[lp];
    d.k = g.m;
    if (!pl.lowrank) d.Rinv = pc->Rinv[pidx[lp]];
    // split of A v_top over column chunks: about kWideBlocks blocks over the batch
    const int64_t nrb = cdiv(g.m, pl.rbN);
    int64_t nch = std::max<int64_t>(1, tl.blocks / std::max<int64_t>(1, rowblocks));
    nch = std::min<int64_t>(nch, cdiv(g.n, 32));
    const int64_t cch = cdiv(cdiv(g.n, nch), 32) * 32;
    nch = cdiv(g.n, cch);
    d.cchunk = cch;
    d.nchN = int32_t(nch);
    d.pnOff = pl.totPN;
    for (int64_t ch = 0; ch < nch; ++ch)
      for (int64_t rb = 0; rb < nrb; ++rb) pl.itNs.push_back({lp, int32_t(rb), int32_t(ch), 0});
    // A^T y over all m rows in one chunk
    d.rchunk = cdiv(g.m, 32) * 32;
    d.nchT = 1;
    d.ptOff = pl.totPT;
    for (int64_t cb = 0; cb < cdiv(g.n, pl.cbT); ++cb) pl.itT.push_back({lp, int32_t(cb), 0, 0});
    // beta partials from the transposed triangular product, alpha partials from k_wide_v
    d.nblkN = int32_t(cdiv(g.m, 4 * pl.cpw));
    if (pl.lowrank) d.nblkN = lowrank_items(pc, pidx[lp], lp, lsel, pl.NC, pl.lr, d);
    d.nblkB = 0;
    d.pnN = pl.nbN;
    d.nblkQ = int32_t(cdiv(g.n, BLK / pl.NC) + cdiv(g.m, BLK / pl.NC));   // k_wide_v blocks
    d.pnQ = pl.nbQ;
    if (!pl.lowrank) {
      for (int i = 0; i < N; ++i)
        for (int b = 0; b < d.nblkN; ++b) pl.itQ.push_back({lp, b, 0, lp * N + i});
      for (int i = 0; i < N; ++i)
        for (int64_t b = 0; b < cdiv(g.m, 16); ++b) pl.itM.push_back({lp, int32_t(b), 0, lp * N + i});
    }
    for (int64_t b = 0; b < cdiv(g.m, BLK / pl.NC); ++b) pl.itR.push_back({lp, int32_t(b), 0, 0});
    for (int b = 0; b < d.nblkQ; ++b) pl.itV.push_back({lp, b, 0, 0});
    for (int64_t b = 0; b < cdiv(g.m, BLK); ++b) pl.itH.push_back({lp, int32_t(b), 0, 0});
    pl.totL += g.n;
    pl.totS += g.m;
    pl.totPN += nch * g.m;
    pl.totPT += g.n;
    pl.nbN += d.nblkN;
    pl.nbQ += d.nblkQ;
    pl.P.push_back(d);
  }
  // The triangular products' blocks differ in length (block b of R^{-T} t reads
  // (b + 1) blocks of rows, row block b of R^{-1} q reads k - 16 b columns):
  // dispatch the longest first so the short ones fill the tail.
  auto q_work = [&](const Item& it) { return (int64_t(it.blk) + 1) * 4 * pl.cpw; };
  auto m_work = [&](const Item& it) { return pl.P[size_t(it.p)].k - 16 * int64_t(it.blk); };
  std::stable_sort(pl.itQ.begin(), pl.itQ.end(),
                   [&](const Item& a, const Item& b) { return q_work(a) > q_work(b); });
  std::stable_sort(pl.itM.begin(), pl.itM.end(),
                   [&](const Item& a, const Item& b) { return m_work(a) > m_work(b); });
  pl.J = np * N;
}

void take_wbufs(Arena& a, const WPlan& pl, size_t tc, WBufs& b) {
  const size_t N = size_t(pl.N);
  b.P = a.take<DevProb>(pl.P.size());
  b.itNs = a.take<Item>(pl.itNs.size());
  b.itT = a.take<Item>(pl.itT.size());
  b.itQ = a.take<Item>(pl.itQ.size());
  b.itM = a.take<Item>(pl.itM.size());
  b.itR = a.take<Item>(pl.itR.size());
  b.itV = a.take<Item>(pl.itV.size());
  b.itH = a.take<Item>(pl.itH.size());
  take_lr(a, pl.lr, b.lr);
  b.sc = a.take<Scal>(pl.J);
  b.partN = a.take<char>(size_t(pl.totPN) * N * tc);
  b.partT = a.take<char>(size_t(pl.totPT) * N * tc);
  b.vt = a.take<double>(size_t(pl.totL) * N);
  b.dt = a.take<double>(size_t(pl.totL) * N);
  b.xt = a.take<double>(size_t(pl.totL) * N);
  b.u = a.take<double>(size_t(pl.totS) * N);
  b.q = a.take<double>(size_t(pl.totS) * N);
  b.y = a.take<double>(size_t(pl.totS) * N);
  b.y32 = a.take<float>(size_t(pl.totS) * N);
  b.w32 = a.take<float>(size_t(pl.totL) * N);
  b.vb = a.take<double>(size_t(pl.totS) * N);
  b.db = a.take<double>(size_t(pl.totS) * N);
  b.zb = a.take<double>(size_t(pl.totS) * N);
  b.t = a.take<double>(size_t(pl.totS) * N);
  b.pnN = a.take<double>(size_t(pl.nbN) * N);
  b.pnQ = a.take<double>(size_t(pl.nbQ) * N);
  b.cnt = a.take<int32_t>(1);
  b.Xp = a.take<double*>(pl.P.size());
  b.lams = a.take<double>(pl.J);
  b.pre = a.take<int32_t>(pl.J);
  b.jmap = a.take<int32_t>(pl.J);
  b.lidx = a.take<int32_t>(pl.J);
}

int upload_wplan(const WPlan& pl, const WBufs& b, const tik_precond_s* pc, double* const* X,
                 std::vector<std::vector<char>>& keep, hipStream_t st) {
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!bytes) return TIK_OK;
    keep.emplace_back(static_cast<const char*>(src), static_cast<const char*>(src) + bytes);
    TIK_HIP(hipMemcpyAsync(dst, keep.back().data(), bytes, hipMemcpyHostToDevice, st));
    return TIK_OK;
  };
  std::vector<DevProb> P = pl.P;
  for (auto& d : P) d.live = b.cnt;
  TIK_HIP(hipMemsetAsync(b.cnt, 1, sizeof(int32_t), st));
  TIK_TRY(put(b.P, P.data(), P.size() * sizeof(DevProb)));
  TIK_TRY(put(b.itNs, pl.itNs.data(), pl.itNs.size() * sizeof(Item)));
  TIK_TRY(put(b.itT, pl.itT.data(), pl.itT.size() * sizeof(Item)));
  TIK_TRY(put(b.itQ, pl.itQ.data(), pl.itQ.size() * sizeof(Item)));
  TIK_TRY(put(b.itM, pl.itM.data(), pl.itM.size() * sizeof(Item)));
  TIK_TRY(put(b.itR, pl.itR.data(), pl.itR.size() * sizeof(Item)));
  TIK_TRY(put(b.itV, pl.itV.data(), pl.itV.size() * sizeof(Item)));
  TIK_TRY(put(b.itH, pl.itH.data(), pl.itH.size() * sizeof(Item)));
  TIK_TRY(put(b.lr.itLP, pl.lr.itLP.data(), pl.lr.itLP.size() * sizeof(Item)));
  TIK_TRY(put(b.lr.itLC, pl.lr.itLC.data(), pl.lr.itLC.size() * sizeof(Item)));
  TIK_TRY(put(b.lr.itLE, pl.lr.itLE.data(), pl.lr.itLE.size() * sizeof(Item)));
  TIK_TRY(put(b.lr.itLF, pl.lr.itLF.data(), pl.lr.itLF.size() * sizeof(Item)));
  std::vector<double> lams(pl.J);
  std::vector<int32_t> pre(pl.J), jmap(pl.J), lidx(pl.J);
  std::vector<double*> xp(pl.P.size());
  for (size_t lp = 0; lp < pl.P.size(); ++lp) {
    const int p = pl.pidx[lp];
    for (int i = 0; i < pl.N; ++i) {
      const int gi = pl.lsel[i];
      lams[lp * pl.N + i] = pc->lams[size_t(p) * pc->N + gi];
      pre[lp * pl.N + i] = pc->status[size_t(p) * pc->N + gi];
      jmap[lp * pl.N + i] = p * pc->N + gi;
      lidx[lp * pl.N + i] = gi;
    }
    xp[lp] = X ? X[p] : nullptr;
  }
  TIK_TRY(put(b.lams, lams.data(), lams.size() * 8));
  TIK_TRY(put(b.pre, pre.data(), pre.size() * 4));
  TIK_TRY(put(b.jmap, jmap.data(), jmap.size() * 4));
  TIK_TRY(put(b.lidx, lidx.data(), lidx.size() * 4));
  TIK_TRY(put(b.Xp, xp.data(), xp.size() * sizeof(double*)));
  return TIK_OK;
}

struct WideIr {
  const int32_t* use;
  const double* h;   // short rows x NF right-hand side
  int NF, l0;
};

template <typename TA, typename TC, int NC>
int wide_products_n(const WPlan& pl, const WBufs& b, const double* W, void* part, hipStream_t st) {
  ProfScope ps("gemm_n", st);
  constexpr bool a32 = std::is_same<TA, float>::value, c32 = std::is_same<TC, float>::value;
  if (NC >= 16) {
    if (c32) TIK_TRY(vec_to_f32(W, int64_t(pl.totL) * pl.N, b.w32, st));
    return launch_gemm_n_mfma(a32, c32, NC, 2, pl.rbN, b.P, b.itNs, int(pl.itNs.size()), pl.N,
                              c32 ? static_cast<const void*>(b.w32) : static_cast<const void*>(W), part,
                              nullptr, b.sc, nullptr, st);
  }
  if (NC >= 8)
    hipLaunchKernelGGL((k_gemm_n<TA, TC, NC, 256, 1, 2>), dim3(unsigned(pl.itNs.size())), dim3(BLK),
                       0, st, b.P, b.itNs, pl.N, W, static_cast<TC*>(part), nullptr, b.sc, nullptr);
  else
    hipLaunchKernelGGL((k_gemm_n<TA, TC, NC, 64, 4, 2>), dim3(unsigned(pl.itNs.size())), dim3(BLK),
                       0, st, b.P, b.itNs, pl.N, W, static_cast<TC*>(part), nullptr, b.sc, nullptr);
  TIK_LAUNCHED("k_gemm_n (split)");
  return TIK_OK;
}

template <typename TA, typename TC, int NC>
int wide_products_t(const WPlan& pl, const WBufs& b, const double* U, void* part, hipStream_t st) {
  ProfScope ps("gemm_t", st);
  constexpr bool a32 = std::is_same<TA, float>::value, c32 = std::is_same<TC, float>::value;
  if (NC >= 16 && c32 && U == b.y) {
    // FP32 products: read y once as FP32 (every column block re-reads it)
    TIK_TRY(vec_to_f32(b.y, int64_t(pl.totS) * pl.N, b.y32, st));
    return launch_gemm_t_mfma(a32, c32, 0, NC, pl.cbT, b.P, b.itT, int(pl.itT.size()), pl.N, b.y32, part,
                              st);
  }
  if (NC >= 16)
    return launch_gemm_t_mfma(a32, c32, 1, NC, pl.cbT, b.P, b.itT, int(pl.itT.size()), pl.N, U, part, st);
  hipLaunchKernelGGL((k_gemm_t<TA, TC, double, NC>), dim3(unsigned(pl.itT.size())), dim3(BLK), 0, st,
                     b.P, b.itT, pl.N, U, int64_t(pl.N), static_cast<TC*>(part));
  TIK_LAUNCHED("k_gemm_t");
  return TIK_OK;
}

template <typename TA, typename TC, int NC>
int wide_v_steps(const WPlan& pl, const WBufs& b, hipStream_t st, bool init, double tol, int maxit) {
  if (pl.lowrank) {
    ProfScope ps("lr_apply", st);
    TIK_TRY(launch_lr_apply(pl.NC, 1, 0, b.P, lr_items(pl.lr, b.lr), pl.N, b.q, lr_bufs(b.lr),
                            b.q, b.u, b.y, nullptr, nullptr, b.sc, nullptr, 0, st));
  } else {
    ProfScope ps("trmv", st);
    hipLaunchKernelGGL(k_trmv<true>, dim3(unsigned(pl.itM.size())), dim3(BLK), 0, st, b.P, b.itM,
                       pl.N, b.q, b.u, b.y, static_cast<double*>(nullptr),
                       static_cast<double*>(nullptr), b.sc, 0);
    TIK_LAUNCHED("k_trmv");
  }
  TIK_TRY((wide_products_t<TA, TC, NC>(pl, b, b.y, b.partT, st)));
  {
    ProfScope ps("vec", st);
    hipLaunchKernelGGL(k_wide_v<TC>, dim3(unsigned(pl.itV.size())), dim3(BLK), 0, st, b.P, b.itV,
                       pl.N, ilog2(pl.NC), static_cast<const TC*>(b.partT), b.y, b.vt, b.vb, b.sc,
                       b.pnQ);
    TIK_LAUNCHED("k_wide_v");
    hipLaunchKernelGGL(k_fin_alpha, dim3(unsigned(pl.J)), dim3(BLK), 0, st, b.P, pl.N, b.pnQ, b.sc,
                       init ? 1 : 0, tol, maxit);
    TIK_LAUNCHED("k_fin_alpha");
    hipLaunchKernelGGL(k_wide_upd, dim3(unsigned(pl.itV.size())), dim3(BLK), 0, st, b.P, b.itV,
                       pl.N, ilog2(pl.NC), b.vt, b.dt, b.xt, b.vb, b.db, b.zb, b.sc, init ? 1 : 0);
    TIK_LAUNCHED("k_wide_upd");
  }
  return TIK_OK;
}

template <int CPW>
int wide_u_tr(const WPlan& pl, const WBufs& b, hipStream_t st) {
  hipLaunchKernelGGL((k_trmv_t<CPW, true>), dim3(unsigned(pl.itQ.size())), dim3(BLK), 0, st, b.P,
                     b.itQ, pl.N, b.t, b.u, b.q, b.sc, b.pnN);
  TIK_LAUNCHED("k_trmv_t");
  return TIK_OK;
}

int wide_u_steps(const WPlan& pl, const WBufs& b, hipStream_t st, bool init) {
  if (pl.lowrank) {
    ProfScope ps("lr_apply", st);
    TIK_TRY(launch_lr_apply(pl.NC, 0, 0, b.P, lr_items(pl.lr, b.lr), pl.N, b.t, lr_bufs(b.lr),
                            b.q, b.u, nullptr, nullptr, nullptr, b.sc, b.pnN, 0, st));
  } else {
    ProfScope ps("trmv_t", st);
    TIK_TRY(pl.cpw == 16 ? wide_u_tr<16>(pl, b, st) : wide_u_tr<4>(pl, b, st));
  }
  ProfScope ps("vec", st);
  hipLaunchKernelGGL(k_fin_beta, dim3(unsigned(pl.J)), dim3(BLK), 0, st, b.P, pl.N, b.pnN,
                     static_cast<const double*>(nullptr), b.sc, init ? 1 : 0,
                     static_cast<const double*>(nullptr), 0);
  TIK_LAUNCHED("k_fin_beta");
  return TIK_OK;
}

template <typename TA, typename TC, int NC>
int run_core_wide(const WPlan& pl, const WBufs& b, double tol, int maxit, hipStream_t st,
                  const WideIr* ir) {
  hipLaunchKernelGGL(k_scal_init, dim3(unsigned(cdiv(pl.J, 256))), dim3(256), 0, st, b.sc, pl.J,
                     pl.N, b.lams, b.pre, b.lidx);
  TIK_LAUNCHED("k_scal_init");
  const size_t S = size_t(pl.totS) * pl.N, L = size_t(pl.totL) * pl.N;
  TIK_HIP(hipMemsetAsync(b.u, 0, S * 8, st));
  TIK_HIP(hipMemsetAsync(b.vb, 0, S * 8, st));
  TIK_HIP(hipMemsetAsync(b.vt, 0, L * 8, st));
  {
    ProfScope ps("vec", st);
    hipLaunchKernelGGL(k_wide_init_h, dim3(unsigned(pl.itH.size())), dim3(BLK), 0, st, b.P, b.itH,
                       pl.N, ir ? ir->NF : 1, ir ? ir->l0 : 0, b.sc, ir ? ir->use : nullptr,
                       ir ? ir->h : nullptr, b.t);
    TIK_LAUNCHED("k_wide_init_h");
  }
  TIK_TRY(wide_u_steps(pl, b, st, true));
  TIK_TRY((wide_v_steps<TA, TC, NC>(pl, b, st, true, tol, maxit)));
  auto body = [&](hipStream_t s) -> int {
    TIK_TRY((wide_products_n<TA, TC, NC>(pl, b, b.vt, b.partN, s)));
    {
      ProfScope ps("vec", s);
      hipLaunchKernelGGL((k_wide_h<TC, NC, 0>), dim3(unsigned(pl.itR.size())), dim3(BLK), 0, s,
                         b.P, b.itR, pl.N, static_cast<const TC*>(b.partN), b.vb, b.sc, b.t);
      TIK_LAUNCHED("k_wide_h");
    }
    TIK_TRY(wide_u_steps(pl, b, s, false));
    return wide_v_steps<TA, TC, NC>(pl, b, s, false, tol, maxit);
  };
  return iterate(body, b.sc, pl.J, b.cnt, maxit, st);
}

template <typename TA, typename TC>
int run_core_wide_nc(const WPlan& pl, const WBufs& b, double tol, int maxit, hipStream_t st,
                     const WideIr* ir) {
  switch (pl.NC) {
    case 1: return run_core_wide<TA, TC, 1>(pl, b, tol, maxit, st, ir);
    case 2: return run_core_wide<TA, TC, 2>(pl, b, tol, maxit, st, ir);
    case 4: return run_core_wide<TA, TC, 4>(pl, b, tol, maxit, st, ir);
    case 8: return run_core_wide<TA, TC, 8>(pl, b, tol, maxit, st, ir);
    case 16: return run_core_wide<TA, TC, 16>(pl, b, tol, maxit, st, ir);
    case 32: return run_core_wide<TA, TC, 32>(pl, b, tol, maxit, st, ir);
  }
  set_error("internal: lambda batch wider than 32");
  return TIK_ENOTSUP;
}

int wide_write(const WPlan& pl, const WBufs& b, int32_t* iters, int32_t* status, double* relres,
               hipStream_t st) {
  int64_t maxn = 0;
  for (auto& d : pl.P) maxn = std::max(maxn, d.n);
  hipLaunchKernelGGL(k_wide_write, dim3(unsigned(std::min<int64_t>(cdiv(maxn, 256), 4096)), unsigned(pl.J)),
                     dim3(256), 0, st, b.P, pl.N, b.xt, b.sc, b.Xp, b.jmap, iters, status, relres);
  TIK_LAUNCHED("k_wide_write");
  return TIK_OK;
}

// ---- dual refinement for wide problems (mixed mode)
// (A A^T + lam I) y = b refined in FP64 with h = b - A x - lam y, x = A^T y;
// the inner minimum-norm solve of [A sqrt(lam) I] z = h gives dy = z_bot / sqrt(lam).
__global__ void k_wide_ir_update(const DevProb* __restrict__ P, int N, int NF, int l0,
                                 const Scal* __restrict__ sc, const int32_t* __restrict__ use,
                                 const double* __restrict__ zb, double* __restrict__ yd) {
  const int j = blockIdx.y, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  const Scal& S = sc[j];
  const bool ok = use[j] && (S.status == TIK_ST_CONVERGED || S.status == TIK_ST_MAXIT);
  if (!ok) return;
  const double isq = 1.0 / S.sqlam;
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < pr.m;
       r += int64_t(gridDim.x) * blockDim.x)
    yd[(pr.irS + r) * NF + (S.li - l0)] += zb[(pr.offS + r) * N + i] * isq;
}

// squared norms of the inner x (the correction of A^T y) and of x + dx, per refinement column
__global__ void __launch_bounds__(BLK) k_wide_ir_norms(const DevProb* __restrict__ P, int N, int NF,
                                                       int l0, const Scal* __restrict__ sc,
                                                       const int32_t* __restrict__ use,
                                                       const double* __restrict__ xin,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ nrm) {
  __shared__ double red[4];
  const int j = blockIdx.x, p = j / N, i = j % N;
  const DevProb& pr = P[p];
  const Scal& S = sc[j];
  const int col = S.li - l0;
  double sd = 0.0, sx = 0.0;
  for (int64_t c = threadIdx.x; c < pr.n; c += BLK) {
    const double d = xin[(pr.offL + c) * N + i];
    const double nx = (x ? x[(pr.irL + c) * NF + col] : 0.0) + d;
    sd += d * d;
    sx += nx * nx;
  }
  const double td = block_sum(sd, red);
  const double tx = block_sum(sx, red);
  if (threadIdx.x == 0 && use[j]) {
    nrm[2 * (pr.gp * NF + col)] = td;
    nrm[2 * (pr.gp * NF + col) + 1] = tx;
  }
}

__global__ void k_wide_ir_write(const DevProb* __restrict__ P, int NF, const double* __restrict__ x,
                                const int32_t* __restrict__ ok, double* const* __restrict__ Xout,
                                int32_t l0) {
  const int j = blockIdx.y, p = j / NF, i = j % NF;
  const DevProb& pr = P[p];
  if (!ok[j]) return;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < pr.n;
       c += int64_t(gridDim.x) * blockDim.x)
    Xout[p][c + int64_t(l0 + i) * pr.n] = x[(pr.offL + c) * NF + i];
}

__global__ void k_ir_stats_wide(const DevProb* __restrict__ P, int J, int N, int NF, int l0,
                                const Scal* __restrict__ sc, const int32_t* __restrict__ use,
                                int32_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int p = j / N;
  const Scal& S = sc[j];
  const int g = P[p].gp * NF + (S.li - l0);
  out[2 * g] = use[j] ? S.iters : 0;
  out[2 * g + 1] = use[j] ? S.status : -1;
}

struct WMixedWs {
  std::vector<float*> A32;
  double *yd, *h, *nrm;
  int32_t *use, *stats, *ok;
  OutRec* rec;
  char *baseF = nullptr, *base32 = nullptr, *base64 = nullptr;
  size_t capF = 0, cap32 = 0, cap64 = 0;
  bool converted = false;
};

size_t wide_mixed_layout(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, Arena& a,
                         WMixedWs& w) {
  std::vector<int> ps;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  const int NF = std::min(32, pc->N);
  std::vector<int> ls;
  all_lambdas(0, NF, ls);
  WPlan pl;
  make_plan_wide(p, pc, ps, ls, pl);
  w.A32.assign(size_t(nprob), nullptr);
  for (int k = 0; k < nprob; ++k)
    if (p[k].a_dtype == TIK_F64) w.A32[k] = a.take<float>(size_t(p[k].m) * size_t(p[k].n));
  w.yd = a.take<double>(size_t(pl.totS) * NF);
  w.h = a.take<double>(size_t(pl.totS) * NF);
  w.nrm = a.take<double>(2 * size_t(pl.J));
  w.use = a.take<int32_t>(pl.J);
  w.stats = a.take<int32_t>(2 * size_t(pl.J));
  w.ok = a.take<int32_t>(pl.J);
  w.rec = a.take<OutRec>(pl.J);
  std::vector<WPlan> subs;
  for (int ng : subset_sizes(NF)) {
    std::vector<int> sub;
    all_lambdas(0, ng, sub);
    subs.emplace_back();
    make_plan_wide(p, pc, ps, sub, subs.back());
  }
  auto region = [&](size_t tc, char*& base, size_t& cap) {
    cap = 0;
    for (const WPlan& q : subs) {
      Arena m;
      WBufs b;
      take_wbufs(m, q, tc, b);
      cap = std::max(cap, m.used + 256);
    }
    base = a.take<char>(cap);
  };
  region(sizeof(double), w.baseF, w.capF);
  region(sizeof(float), w.base32, w.cap32);
  region(sizeof(double), w.base64, w.cap64);
  return a.used;
}

template <typename TA64>
int wide_mixed_group(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, WMixedWs& w,
                     int l0, int NF, double tol, int maxit, double* const* X, int32_t* iters,
                     int32_t* status, double* relres, hipStream_t st) {
  std::vector<int> ps;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  std::vector<int> lsel;
  all_lambdas(l0, NF, lsel);
  std::vector<std::vector<char>> keep;
  // hard lambdas: the whole group in FP64 (same rule as for tall problems)
  bool any_hard = false;
  for (int i = 0; i < NF; ++i)
    for (int k = 0; k < nprob; ++k) {
      const double lam = pc->lams[size_t(k) * pc->N + l0 + i];
      any_hard |= 12.0 * std::sqrt((pc->cnorm[k] + lam) / lam) * std::ldexp(1.0, -24) > 0.25;
    }
  if (any_hard) {
    WPlan ph;
    make_plan_wide(p, pc, ps, lsel, ph);
    Arena ah;
    ah.base = w.base64;
    ah.cap = w.cap64;
    WBufs bh;
    take_wbufs(ah, ph, sizeof(double), bh);
    TIK_TRY(upload_wplan(ph, bh, pc, X, keep, st));
    note_split(0, ph.J);
    TIK_TRY((run_core_wide_nc<TA64, double>(ph, bh, std::max(1e-3 * tol, 1e-14), maxit, st, nullptr)));
    TIK_TRY(wide_write(ph, bh, iters, status, relres, st));
    TIK_HIP(hipStreamSynchronize(st));
    return TIK_OK;
  }
  // FP64 plan over all lambdas of the group: A^T y and h = b - A x - lam y
  WPlan pf;
  make_plan_wide(p, pc, ps, lsel, pf);
  Arena af;
  af.base = w.baseF;
  af.cap = w.capF;
  WBufs bf;
  take_wbufs(af, pf, sizeof(double), bf);
  TIK_TRY(upload_wplan(pf, bf, pc, nullptr, keep, st));
  hipLaunchKernelGGL(k_scal_init, dim3(unsigned(cdiv(pf.J, 256))), dim3(256), 0, st, bf.sc, pf.J,
                     pf.N, bf.lams, bf.pre, bf.lidx);
  TIK_LAUNCHED("k_scal_init");
  const int J = pf.J;
  note_split(J, 0);
  const size_t S = size_t(pf.totS) * NF;
  TIK_HIP(hipMemsetAsync(w.yd, 0, S * 8, st));
  if (!w.converted) {
    ProfScope ps_("residual", st);
    for (int k = 0; k < nprob; ++k)
      if (w.A32[k]) {
        const int64_t tot = p[k].m * p[k].n;
        hipLaunchKernelGGL(k_to_f32, dim3(unsigned(std::min<int64_t>(cdiv(tot, 256), 65536))),
                           dim3(256), 0, st, static_cast<const double*>(p[k].A), p[k].m, p[k].n,
                           p[k].lda, w.A32[k]);
        TIK_LAUNCHED("k_to_f32");
      }
    w.converted = true;
  }
  std::vector<int32_t> st_h(J, -1), it_h(J, 0);
  std::vector<double> rel_h(J, 0.0), dxrel(J, 1.0);
  std::vector<uint8_t> done(J, 0);
  for (int j = 0; j < J; ++j) {
    const int32_t pre = pc->status[size_t(j / NF) * pc->N + l0 + (j % NF)];
    if (pre != TIK_ST_CONVERGED) {
      st_h[j] = pre;
      done[j] = 1;
    }
  }
  std::vector<const void*> Aov(static_cast<size_t>(nprob));
  std::vector<int64_t> ldo(static_cast<size_t>(nprob));
  for (int k = 0; k < nprob; ++k) {
    Aov[k] = w.A32[k] ? static_cast<const void*>(w.A32[k]) : p[k].A;
    ldo[k] = w.A32[k] ? p[k].m : p[k].lda;
  }
  const double tol32 = std::max(tol, 1e-6);
  const int maxsweep = 12;
  std::vector<double> nrm(2 * size_t(J));
  std::vector<int32_t> stats(2 * size_t(J));
  const double* xcur = nullptr;   // x = A^T y of the current sweep (FP64, in bf.partT)
  for (int sweep = 1; sweep <= maxsweep; ++sweep) {
    std::vector<int> sel;
    std::vector<uint8_t> use(J, 0);
    for (int i = 0; i < NF; ++i) {
      bool act = false;
      for (int k = 0; k < nprob; ++k) act |= !done[k * NF + i];
      if (!act) continue;
      sel.push_back(l0 + i);
      for (int k = 0; k < nprob; ++k)
        if (!done[k * NF + i]) use[k * NF + i] = 1;
    }
    if (sel.empty()) break;
    const double* hr = nullptr;
    if (sweep > 1) {
      // x = A^T y (FP64); h = b - A x - lam y (FP64)
      switch (pf.NC) {
#define WP(nc) case nc: TIK_TRY((wide_products_t<TA64, double, nc>(pf, bf, w.yd, bf.partT, st))); \
                        TIK_TRY((wide_products_n<TA64, double, nc>(pf, bf, static_cast<const double*>(bf.partT), bf.partN, st))); \
                        hipLaunchKernelGGL((k_wide_h<double, nc, 1>), dim3(unsigned(pf.itR.size())), dim3(BLK), 0, st, bf.P, bf.itR, pf.N, static_cast<const double*>(bf.partN), w.yd, bf.sc, w.h); break;
        WP(1) WP(2) WP(4) WP(8) WP(16) WP(32)
#undef WP
      }
      TIK_LAUNCHED("k_wide_h (refinement)");
      hr = w.h;
      xcur = static_cast<const double*>(bf.partT);
    }
    // inner FP32 minimum-norm solve over the selected lambdas, over only the
    // problems with a lambda to correct (the region is sized for all problems;
    // a subset splits its columns finer and may need more partial rows: then
    // it takes them all)
    std::vector<int> pin;
    for (int k = 0; k < nprob; ++k) {
      bool any = false;
      for (int li : sel) any |= use[size_t(k) * NF + size_t(li - l0)] != 0;
      if (any) pin.push_back(k);
    }
    WPlan pl;
    make_plan_wide(p, pc, pin, sel, pl, Aov.data(), ldo.data());
    {
      Arena m;
      WBufs mb;
      take_wbufs(m, pl, sizeof(float), mb);
      if (m.used > w.cap32 && pin.size() < size_t(nprob)) {
        pin = ps;
        make_plan_wide(p, pc, pin, sel, pl, Aov.data(), ldo.data());
      }
    }
    for (size_t lp = 0; lp < pl.P.size(); ++lp) {
      pl.P[lp].a_f32 = 1;
      pl.P[lp].irL = pf.P[size_t(pin[lp])].offL;
      pl.P[lp].irS = pf.P[size_t(pin[lp])].offS;
    }
    Arena ai;
    ai.base = w.base32;
    ai.cap = w.cap32;
    WBufs bi;
    take_wbufs(ai, pl, sizeof(float), bi);
    if (!ai.fits()) {
      set_error("internal: inner plan exceeds its region");
      return TIK_EWORKSPACE;
    }
    TIK_TRY(upload_wplan(pl, bi, pc, nullptr, keep, st));
    std::vector<int32_t> uj(size_t(pl.J));
    for (size_t lp = 0; lp < pin.size(); ++lp)
      for (size_t i = 0; i < sel.size(); ++i)
        uj[lp * sel.size() + i] = use[size_t(pin[lp]) * NF + size_t(sel[i] - l0)];
    keep.emplace_back(reinterpret_cast<const char*>(uj.data()), reinterpret_cast<const char*>(uj.data()) + uj.size() * 4);
    TIK_HIP(hipMemcpyAsync(w.use, keep.back().data(), uj.size() * 4, hipMemcpyHostToDevice, st));
    WideIr ir{w.use, hr, NF, l0};
    TIK_TRY((run_core_wide_nc<float, float>(pl, bi, tol32, maxit, st, hr ? &ir : nullptr)));
    if (!hr) {
      // first sweep solved with b itself: every selected lambda is used
    }
    hipLaunchKernelGGL(k_wide_ir_update, dim3(unsigned(cdiv(pf.P[0].m, 256) + 1), unsigned(pl.J)),
                       dim3(256), 0, st, bi.P, pl.N, NF, l0, bi.sc, w.use, bi.zb, w.yd);
    TIK_LAUNCHED("k_wide_ir_update");
    TIK_HIP(hipMemsetAsync(w.nrm, 0, nrm.size() * 8, st));
    hipLaunchKernelGGL(k_wide_ir_norms, dim3(unsigned(pl.J)), dim3(BLK), 0, st, bi.P, pl.N, NF, l0,
                       bi.sc, w.use, bi.xt, xcur, w.nrm);
    TIK_LAUNCHED("k_wide_ir_norms");
    TIK_HIP(hipMemsetAsync(w.stats, 0xFF, stats.size() * 4, st));
    hipLaunchKernelGGL(k_ir_stats_wide, dim3(unsigned(cdiv(pl.J, 256))), dim3(256), 0, st, bi.P,
                       pl.J, pl.N, NF, l0, bi.sc, w.use, w.stats);
    TIK_LAUNCHED("k_ir_stats_wide");
    TIK_HIP(hipMemcpyAsync(nrm.data(), w.nrm, nrm.size() * 8, hipMemcpyDeviceToHost, st));
    TIK_HIP(hipMemcpyAsync(stats.data(), w.stats, stats.size() * 4, hipMemcpyDeviceToHost, st));
    TIK_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < J; ++j) {
      if (done[j] || !use[j]) continue;
      it_h[j] += std::max(0, stats[2 * j]);
      const int32_t ist = stats[2 * j + 1];
      if (ist == TIK_ST_NOTPD || ist == TIK_ST_NONFINITE) {
        st_h[j] = ist;
        done[j] = 1;
        continue;
      }
      const double nd = std::sqrt(nrm[2 * j]), nx = std::sqrt(nrm[2 * j + 1]);
      if (!std::isfinite(nd) || !std::isfinite(nx)) {
        st_h[j] = TIK_ST_NONFINITE;
        done[j] = 1;
        continue;
      }
      const double rel = nx > 0.0 ? nd / nx : 0.0;
      rel_h[j] = rel;
      // converged as in the tall driver: small correction, or (from the third
      // sweep on) contracting sweeps whose predicted remaining error is a
      // hundred times below tol
      const double r_k = sweep == 1 ? 1.0 : rel / std::max(dxrel[j], 1e-300);
      if (rel <= tol || (sweep >= 3 && r_k < 0.1 && r_k * rel <= 1e-2 * tol)) {
        st_h[j] = TIK_ST_CONVERGED;
        done[j] = 1;
      } else if (sweep >= 3 && rel > 0.9 * dxrel[j]) {
        st_h[j] = TIK_ST_IR_STALL;
        done[j] = 1;
      } else if (sweep == maxsweep) {
        st_h[j] = TIK_ST_MAXIT;
        done[j] = 1;
      }
      dxrel[j] = rel;
    }
  }
  for (int j = 0; j < J; ++j)
    if (!done[j]) st_h[j] = TIK_ST_MAXIT;
  // final x = A^T y in FP64
  switch (pf.NC) {
#define WT(nc) case nc: TIK_TRY((wide_products_t<TA64, double, nc>(pf, bf, w.yd, bf.partT, st))); break;
    WT(1) WT(2) WT(4) WT(8) WT(16) WT(32)
#undef WT
  }
  std::vector<int32_t> okv(J);
  for (int j = 0; j < J; ++j)
    okv[j] = (st_h[j] == TIK_ST_CONVERGED || st_h[j] == TIK_ST_MAXIT || st_h[j] == TIK_ST_IR_STALL) ? 1 : 0;
  keep.emplace_back(reinterpret_cast<const char*>(okv.data()), reinterpret_cast<const char*>(okv.data()) + J * 4);
  TIK_HIP(hipMemcpyAsync(w.ok, keep.back().data(), size_t(J) * 4, hipMemcpyHostToDevice, st));
  std::vector<double*> xp(static_cast<size_t>(nprob));
  for (int k = 0; k < nprob; ++k) xp[k] = X[k];
  keep.emplace_back(reinterpret_cast<const char*>(xp.data()), reinterpret_cast<const char*>(xp.data()) + xp.size() * sizeof(double*));
  TIK_HIP(hipMemcpyAsync(bf.Xp, keep.back().data(), xp.size() * sizeof(double*), hipMemcpyHostToDevice, st));
  int64_t maxn = 0;
  for (auto& d : pf.P) maxn = std::max(maxn, d.n);
  hipLaunchKernelGGL(k_wide_ir_write, dim3(unsigned(std::min<int64_t>(cdiv(maxn, 256), 4096)), unsigned(J)),
                     dim3(256), 0, st, bf.P, NF, static_cast<const double*>(bf.partT), w.ok, bf.Xp, l0);
  TIK_LAUNCHED("k_wide_ir_write");
  std::vector<OutRec> recs;
  for (int j = 0; j < J; ++j)
    recs.push_back(OutRec{int64_t(j / NF) * pc->N + l0 + (j % NF), it_h[j], st_h[j], rel_h[j]});
  TIK_TRY(scatter_outs(recs, w.rec, iters, status, relres, keep, st));
  TIK_HIP(hipStreamSynchronize(st));
  return TIK_OK;
}

int wide_bytes(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode,
               size_t* bytes) {
  if (mode == TIK_MIXED_BATCHED) {
    Arena a;
    WMixedWs w;
    *bytes = wide_mixed_layout(p, nprob, pc, a, w) + 256;
    return TIK_OK;
  }
  std::vector<std::vector<int>> gp, gl;
  groups_for(pc, nprob, mode, gp, gl);
  size_t best = 0;
  for (size_t g = 0; g < gp.size(); ++g) {
    WPlan pl;
    make_plan_wide(p, pc, gp[g], gl[g], pl);
    Arena a;
    WBufs b;
    take_wbufs(a, pl, sizeof(double), b);
    best = std::max(best, a.used);
  }
  *bytes = best + 256;
  return TIK_OK;
}

int wide_run(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode, double tol,
             int32_t maxit, double* const* X, int32_t* iters, int32_t* status, double* relres,
             void* dws, size_t dws_bytes, hipStream_t st) {
  const bool f32 = p[0].a_dtype == TIK_F32;
  if (mode == TIK_MIXED_BATCHED) {
    Arena a;
    a.base = static_cast<char*>(dws);
    a.cap = dws_bytes;
    WMixedWs w;
    wide_mixed_layout(p, nprob, pc, a, w);
    if (!a.fits()) {
      set_error("tik_lsqr_batch: workspace too small");
      return TIK_EWORKSPACE;
    }
    for (int l0 = 0; l0 < pc->N; l0 += 32) {
      const int NF = std::min(32, pc->N - l0);
      if (f32)
        TIK_TRY(wide_mixed_group<float>(p, nprob, pc, w, l0, NF, tol, maxit, X, iters, status, relres, st));
      else
        TIK_TRY(wide_mixed_group<double>(p, nprob, pc, w, l0, NF, tol, maxit, X, iters, status, relres, st));
    }
    return TIK_OK;
  }
  std::vector<std::vector<int>> gp, gl;
  groups_for(pc, nprob, mode, gp, gl);
  for (size_t g = 0; g < gp.size(); ++g) {
    WPlan pl;
    make_plan_wide(p, pc, gp[g], gl[g], pl);
    Arena a;
    a.base = static_cast<char*>(dws);
    a.cap = dws_bytes;
    WBufs b;
    take_wbufs(a, pl, sizeof(double), b);
    if (!a.fits()) {
      set_error("tik_lsqr_batch: workspace too small");
      return TIK_EWORKSPACE;
    }
    std::vector<std::vector<char>> keep;
    TIK_TRY(upload_wplan(pl, b, pc, X, keep, st));
    note_split(0, pl.J);
    if (f32)
      TIK_TRY((run_core_wide_nc<float, double>(pl, b, tol, maxit, st, nullptr)));
    else
      TIK_TRY((run_core_wide_nc<double, double>(pl, b, tol, maxit, st, nullptr)));
    TIK_TRY(wide_write(pl, b, iters, status, relres, st));
    TIK_HIP(hipStreamSynchronize(st));
    if (option_record_times()) {
      std::vector<Scal> hs(static_cast<size_t>(pl.J));
      TIK_HIP(hipMemcpyAsync(hs.data(), b.sc, hs.size() * sizeof(Scal), hipMemcpyDeviceToHost, st));
      TIK_HIP(hipStreamSynchronize(st));
      times_note(hs.data(), pl.J, pl.N, pl.pidx, pl.lsel, pc->N, st);
    }
  }
  return TIK_OK;
}

}  // namespace

// ---------------------------------------------------------------- tuning ----
// Candidate launch shapes: rows per gemm_n block x columns per gemm_t block x
// product-block target (only the target applies to the few-lambda kernels).
std::vector<Tile> tile_candidates(int nc) {
  std::vector<Tile> c;
  const int blocks[] = {1024, 2048, 4096};
  if (nc < 16) {
    for (int b : blocks) c.push_back(Tile{0, 0, b});
    return c;
  }
  for (int r : {128, 256})
    for (int t : {64, 128})
      for (int b : blocks) c.push_back(Tile{r, t, b});
  return c;
}

struct OverrideScope {
  explicit OverrideScope(const Tile* t) { t_tile_override = t; }
  ~OverrideScope() { t_tile_override = nullptr; }
};

// Time `iters` batched FP64 LSQR iterations of the first (up to 32) lambdas of
// every problem with each candidate and keep the fastest for the class.
int tune_class(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t iters, void* dws,
               size_t dws_bytes, hipStream_t st, int* best_out, double* best_ms_out, double* default_ms_out) {
  tile_autoload();   // a later first load must not replace what this call stores
  std::vector<int> ps, ls;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  for (int i = 0; i < std::min(32, pc->N); ++i) ls.push_back(i);
  const bool wide = pc->wide;
  const bool f32 = p[0].a_dtype == TIK_F32;
  const int nc = pick_nc(int(ls.size()));
  const std::vector<Tile> cand = tile_candidates(nc);
  hipEvent_t e0, e1;
  TIK_HIP(hipEventCreate(&e0));
  TIK_HIP(hipEventCreate(&e1));
  double best = 1e300, dflt = -1.0;
  int bi = -1;
  int rc = TIK_OK;
  const Tile def = tile_default(wide ? 1 : 0);
  for (size_t ci = 0; ci < cand.size() && rc == TIK_OK; ++ci) {
    Tile t = cand[ci];
    if (nc < 16) {
      t.rbN = def.rbN;
      t.cbT = def.cbT;
    }
    OverrideScope ov(&t);
    double ms_min = 1e300;
    for (int rep = 0; rep < 2 && rc == TIK_OK; ++rep) {
      std::vector<std::vector<char>> keep;
      Arena a;
      a.base = static_cast<char*>(dws);
      a.cap = dws_bytes;
      if (wide) {
        WPlan pl;
        make_plan_wide(p, pc, ps, ls, pl);
        WBufs b;
        take_wbufs(a, pl, sizeof(double), b);
        if (!a.fits()) { set_error("tik_tune: workspace too small"); rc = TIK_EWORKSPACE; break; }
        if ((rc = upload_wplan(pl, b, pc, nullptr, keep, st)) != TIK_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = TIK_EHIP; break; }
        rc = f32 ? run_core_wide_nc<float, double>(pl, b, 0.0, iters, st, nullptr)
                 : run_core_wide_nc<double, double>(pl, b, 0.0, iters, st, nullptr);
      } else {
        Plan pl;
        make_plan(p, pc, ps, ls, pl);
        Bufs b;
        take_bufs(a, pl, sizeof(double), b);
        if (!a.fits()) { set_error("tik_tune: workspace too small"); rc = TIK_EWORKSPACE; break; }
        if ((rc = upload_plan(pl, b, pc, nullptr, keep, st)) != TIK_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = TIK_EHIP; break; }
        rc = f32 ? run_core_nc<float, double>(pl, b, 0.0, iters, st, nullptr)
                 : run_core_nc<double, double>(pl, b, 0.0, iters, st, nullptr);
      }
      if (rc != TIK_OK) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = TIK_EHIP; break; }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = TIK_EHIP; break; }
      if (rep > 0) ms_min = std::min(ms_min, double(ms));   // the first run captures its graph
    }
    if (rc != TIK_OK) break;
    if (t.rbN == def.rbN && t.cbT == def.cbT && t.blocks == def.blocks) dflt = ms_min;
    if (ms_min < best) {
      best = ms_min;
      bi = int(ci);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TIK_TRY(rc);
  Tile t = cand[size_t(bi)];
  if (nc < 16) {
    t.rbN = def.rbN;
    t.cbT = def.cbT;
  }
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tiles[tile_key(wide ? 1 : 0, p, ps, f32, nc)] = t;
  }
  if (best_out) {
    best_out[0] = t.rbN;
    best_out[1] = t.cbT;
    best_out[2] = t.blocks;
  }
  if (best_ms_out) *best_ms_out = best;
  if (default_ms_out) *default_ms_out = dflt;
  return TIK_OK;
}

int tune_bytes(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, size_t* bytes) {
  std::vector<int> ps, ls;
  for (int k = 0; k < nprob; ++k) ps.push_back(k);
  for (int i = 0; i < std::min(32, pc->N); ++i) ls.push_back(i);
  size_t need = 0;
  for (const Tile& c : tile_candidates(pick_nc(int(ls.size())))) {
    Tile t = c;
    const Tile def = tile_default(pc->wide ? 1 : 0);
    if (t.rbN == 0) {
      t.rbN = def.rbN;
      t.cbT = def.cbT;
    }
    OverrideScope ov(&t);
    Arena a;
    if (pc->wide) {
      WPlan pl;
      make_plan_wide(p, pc, ps, ls, pl);
      WBufs b;
      take_wbufs(a, pl, sizeof(double), b);
    } else {
      Plan pl;
      make_plan(p, pc, ps, ls, pl);
      Bufs b;
      take_bufs(a, pl, sizeof(double), b);
    }
    need = std::max(need, a.used + 256);
  }
  *bytes = need;
  return TIK_OK;
}

// The mixed drivers solve a group of lambdas by batched FP64 LSQR when FP32
// products cannot carry one of its lambdas (12 kappa(B) u_32 > 0.25, kappa(B)^2
// bounded by (||C|| + lambda) / lambda).  When that holds for every group, a
// mixed call is batched FP64 at the refinement's inner tolerance: it runs as
// such, without planning the refinement's workspace.
static bool all_groups_fp64(int32_t nprob, const tik_precond_s* pc) {
  for (int l0 = 0; l0 < pc->N; l0 += 32) {
    bool any = false;
    for (int i = l0; i < std::min(pc->N, l0 + 32); ++i)
      for (int k = 0; k < nprob; ++k) {
        const double lam = pc->lams[size_t(k) * pc->N + i];
        any |= 12.0 * std::sqrt((pc->cnorm[k] + lam) / lam) * std::ldexp(1.0, -24) > 0.25;
      }
    if (!any) return false;
  }
  return true;
}

int lsqr_bytes(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode,
               size_t* bytes) {
  if (mode == TIK_MIXED_BATCHED && all_groups_fp64(nprob, pc)) mode = TIK_F64_BATCHED;
  if (pc->wide) return wide_bytes(p, nprob, pc, mode, bytes);
  if (mode == TIK_MIXED_BATCHED) {
    Arena a;
    MixedWs w;
    *bytes = mixed_layout(p, nprob, pc, a, w) + 256;
    return TIK_OK;
  }
  std::vector<std::vector<int>> gp, gl;
  groups_for(pc, nprob, mode, gp, gl);
  size_t best = 0;
  const size_t tc = mode == TIK_MIXED_BATCHED ? sizeof(float) : sizeof(double);
  for (size_t g = 0; g < gp.size(); ++g) {
    Plan pl;
    make_plan(p, pc, gp[g], gl[g], pl);
    Arena a;
    Bufs b;
    take_bufs(a, pl, tc, b);
    best = std::max(best, a.used);
  }
  *bytes = best + 256;
  return TIK_OK;
}

int lsqr_run(const tik_problem* p, int32_t nprob, const tik_precond_s* pc, int32_t mode,
             double tol, int32_t maxit, double* const* X, int32_t* iters, int32_t* status,
             double* relres, void* dws, size_t dws_bytes, hipStream_t st) {
  if (mode == TIK_MIXED_BATCHED && all_groups_fp64(nprob, pc)) {
    mode = TIK_F64_BATCHED;
    tol = std::max(1e-3 * tol, 1e-14);      // the mixed drivers' tolerance for such groups
  }
  if (pc->wide)
    return wide_run(p, nprob, pc, mode, tol, maxit, X, iters, status, relres, dws, dws_bytes, st);
  if (mode == TIK_MIXED_BATCHED)
    return mixed_run(p, nprob, pc, tol, maxit, X, iters, status, relres, dws, dws_bytes, st);
  std::vector<std::vector<int>> gp, gl;
  groups_for(pc, nprob, mode, gp, gl);
  const bool f32 = p[0].a_dtype == TIK_F32;
  for (size_t g = 0; g < gp.size(); ++g) {
    Plan pl;
    make_plan(p, pc, gp[g], gl[g], pl);
    Arena a;
    a.base = static_cast<char*>(dws);
    a.cap = dws_bytes;
    Bufs b;
    take_bufs(a, pl, sizeof(double), b);
    if (!a.fits()) {
      set_error("tik_lsqr_batch: workspace too small");
      return TIK_EWORKSPACE;
    }
    std::vector<std::vector<char>> keep;
    TIK_TRY(upload_plan(pl, b, pc, X, keep, st));
    note_split(0, pl.J);
    if (f32)
      TIK_TRY((run_core_nc<float, double>(pl, b, tol, maxit, st, nullptr)));
    else
      TIK_TRY((run_core_nc<double, double>(pl, b, tol, maxit, st, nullptr)));
    int64_t maxn = 0;
    for (auto& d : pl.P) maxn = std::max(maxn, d.n);
    hipLaunchKernelGGL(k_write_out_map, dim3(unsigned(cdiv(maxn, 256)), unsigned(pl.J)), dim3(256), 0,
                       st, b.P, pl.N, b.x, b.sc, b.Xp, b.jmap, iters, status, relres);
    TIK_LAUNCHED("k_write_out");
    TIK_HIP(hipStreamSynchronize(st));   // staging vectors in `keep` die here
    if (option_record_times()) {
      std::vector<Scal> hs(static_cast<size_t>(pl.J));
      TIK_HIP(hipMemcpyAsync(hs.data(), b.sc, hs.size() * sizeof(Scal), hipMemcpyDeviceToHost, st));
      TIK_HIP(hipStreamSynchronize(st));
      times_note(hs.data(), pl.J, pl.N, pl.pidx, pl.lsel, pc->N, st);
    }
  }
  return TIK_OK;
}

// ------------------------------------------------------ tile persistence ----
// Text format, one class per line:
//   wide a32 nc lm ln lp  rbN cbT blocks
// '#' starts a comment.
int tiles_save(const char* path) {
  tile_autoload();
  FILE* f = std::fopen(path, "w");
  if (!f) {
    set_error(std::string("tik_tune_save: cannot open ") + path);
    return TIK_EINVAL;
  }
  std::fprintf(f, "# libtik launch-shape table: wide a32 nc log2(m) log2(n) problems(0:1,1:<=16,2:more)"
                  "  rows_per_gemm_n_block cols_per_gemm_t_block product_blocks\n");
  std::lock_guard<std::mutex> lk(g_tile_mu);
  for (const auto& kv : g_tiles)
    std::fprintf(f, "%d %d %d %d %d %d  %d %d %d\n", kv.first.wide, kv.first.a32, kv.first.nc, kv.first.lm,
                 kv.first.ln, kv.first.lp, kv.second.rbN, kv.second.cbT, kv.second.blocks);
  std::fclose(f);
  return TIK_OK;
}

static int tiles_read(const char* path, int* loaded);

int tiles_load(const char* path, int* loaded) {
  tile_autoload();   // an explicit file then overrides the automatic one
  return tiles_read(path, loaded);
}

// Merge a table file into the table (all of it, or nothing when a line is malformed).
static int tiles_read(const char* path, int* loaded) {
  FILE* f = std::fopen(path, "r");
  if (!f) {
    set_error(std::string("tik_tune_load: cannot open ") + path);
    return TIK_EINVAL;
  }
  char line[512];
  int n = 0, lineno = 0;
  std::map<TileKey, Tile> add;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    char* h = std::strchr(line, '#');
    if (h) *h = 0;
    if (std::strspn(line, " \t\r\n") == std::strlen(line)) continue;   // blank or comment only
    TileKey k;
    Tile t;
    int used = 0;
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %n", &k.wide, &k.a32, &k.nc, &k.lm, &k.ln,
                                &k.lp, &t.rbN, &t.cbT, &t.blocks, &used);
    const bool whole = got == 9 && line[used] == 0;
    const bool ok = whole && (k.wide == 0 || k.wide == 1) && (k.a32 == 0 || k.a32 == 1) &&
                    (k.nc == 1 || k.nc == 2 || k.nc == 4 || k.nc == 8 || k.nc == 16 || k.nc == 32) &&
                    (t.rbN == 64 || t.rbN == 128 || t.rbN == 256) && (t.cbT == 64 || t.cbT == 128) &&
                    t.blocks >= 64 && t.blocks <= (1 << 16) && k.lp >= 0 && k.lp <= 2;
    if (!ok) {
      std::fclose(f);
      set_error(std::string("tik_tune_load: malformed line ") + std::to_string(lineno) + " in " + path);
      return TIK_EINVAL;
    }
    add[k] = t;
    ++n;
  }
  std::fclose(f);
  std::lock_guard<std::mutex> lk(g_tile_mu);
  for (const auto& kv : add) g_tiles[kv.first] = kv.second;
  if (loaded) *loaded = n;
  return TIK_OK;
}

// tuning.txt beside the library, read once on first use when present
void tile_autoload() {
  std::call_once(g_tile_once, []() {
    Dl_info info;
    if (!dladdr(reinterpret_cast<void*>(&tik_version), &info) || !info.dli_fname) return;
    std::string dir(info.dli_fname);
    const size_t slash = dir.rfind('/');
    dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
    const std::string path = dir + "/tuning.txt";
    if (FILE* f = std::fopen(path.c_str(), "r")) {
      std::fclose(f);
      (void)tiles_read(path.c_str(), nullptr);   // a malformed file leaves the defaults in place
    }
  });
}

const std::string& last_tile() { return t_last_tile; }

}  // namespace tik
