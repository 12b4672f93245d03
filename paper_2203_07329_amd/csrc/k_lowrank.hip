// Low-statistical-dimension preconditioner (Algorithm 3, Section 3.1).
//
// From the short, fat sketch Y = XA (s x n, s <= n) the route needs the
// economy SVD Y = U Sigma V^T (Algorithm 3 step 4) without ever forming a Gram
// matrix:
//   1. Householder QR of Y^T (n x s) in FP64: Y^T = Q1 R1, blocked in panels of
//      32 columns with compact-WY trailing updates (Schreiber & Van Loan).
//      Each panel is factored by two Cholesky QR passes and a reconstruction
//      of its reflectors (a fixed dozen launches), or, where its scaled Gram
//      matrix is nearly singular, column by column (one launch per column).
//   2. A second Householder QR, of R1^T = Q2 R2, so that Y^T = Q1 R2^T Q2^T.
//      The lower triangle L = R2^T has far more nearly orthogonal columns than
//      R1, which cuts the sweeps of the next step by more than half (the QR
//      preconditioning of one-sided Jacobi, Drmac & Veselic 2008).
//   3. One-sided Jacobi (Hestenes) on L: plane rotations orthogonalise its
//      columns, L W = Z Sigma; the normalised columns Z are the left singular
//      vectors of L and their norms the singular values.  Round-robin
//      ordering: every round rotates s/2 disjoint column pairs in parallel.
//   4. Y^T = (Q1 Z) Sigma (Q2 W)^T, so the right singular vectors of Y are
//      V = Q1 Z: the reflectors of step 1 applied to [Z; 0].  Neither W nor Q2
//      is ever formed.
// sd_hat (Section 3.1.2), s_i and S_i (Algorithm 3 steps 5-7) are formed from
// the singular values per lambda.
#include "tik_internal.h"

#include <cmath>

namespace tik {

static constexpr int LR_NB = 32;      // Householder panel width

__device__ __forceinline__ double lr_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ double lr_block_sum(double v, double* red) {
  v = lr_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// Z (n x s, ld n) = Y^T with Y s x n (ld s).
__global__ void k_lr_transpose(const double* __restrict__ Y, int64_t s, int64_t n,
                               double* __restrict__ Z) {
  __shared__ double tile[32][33];
  const int64_t r0 = int64_t(blockIdx.x) * 32, c0 = int64_t(blockIdx.y) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;          // Y(r, c), r < s, c < n
    tile[k][tx] = (r < s && c < n) ? Y[r + c * s] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;          // Z(c, r) = Y(r, c)
    if (c < n && r < s) Z[c + r * n] = tile[tx][k];
  }
}

// dlarfg (as LAPACK defines it) on column c of Z, rows c .. rows-1, given
// sigma = sum of squares of rows c+1 .. rows-1 and alpha = Z[c, c]: beta =
// -sign(alpha) sqrt(alpha^2 + sigma), tau = (beta - alpha) / beta, v = x /
// (alpha - beta) below the diagonal (v_0 = 1 implied).  Thread 0 writes
// Z[c, c] = beta and tau[c] and returns the scale of v in *sh_scale (0: no
// reflection, tau = 0).
__device__ __forceinline__ void lr_house_head(double* col, int64_t c, double alpha, double sigma,
                                              double* tau, double* sh_scale) {
  if (sigma == 0.0) {
    tau[c] = 0.0;
    *sh_scale = 0.0;
  } else {
    const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
    tau[c] = (beta - alpha) / beta;
    *sh_scale = 1.0 / (alpha - beta);
    col[c] = beta;
  }
}

// Rows lo + threadIdx.x + 1024 (u + U i) of a column: U independent loads per
// thread and step.
#define TIK_LR_ROWS(LO, ROWS, BODY)                                                   \
  for (int64_t r0_ = (LO); r0_ < (ROWS); r0_ += 1024 * LR_U) {                        \
    _Pragma("unroll") for (int u_ = 0; u_ < LR_U; ++u_) {                             \
      const int64_t r = r0_ + threadIdx.x + 1024 * u_;                                \
      if (r < (ROWS)) { BODY }                                                        \
    }                                                                                 \
  }
constexpr int LR_U = 4;

// Householder vector of column j of Z (rows x *, ld ldz): dlarfg on rows
// j .. rows-1.  One block of 1024 threads.
__global__ void __launch_bounds__(1024) k_lr_house(double* __restrict__ Z, int64_t ldz, int64_t rows,
                                                   int64_t j, double* __restrict__ tau) {
  __shared__ double red[16];
  __shared__ double sh_scale;
  double* col = Z + j * ldz;
  double ss = 0.0;
  TIK_LR_ROWS(j + 1, rows, { const double x = col[r]; ss += x * x; })
  const double sigma = lr_block_sum<1024>(ss, red);
  if (threadIdx.x == 0) lr_house_head(col, j, col[j], sigma, tau, &sh_scale);
  __syncthreads();
  const double sc = sh_scale;
  if (sc != 0.0) TIK_LR_ROWS(j + 1, rows, { col[r] *= sc; })
}

// Apply H_j = I - tau_j v v^T to the columns j+1 .. j+gridDim.x of Z (one
// block of 1024 threads per column).  With `next`, block 0 (column j+1) then
// forms the Householder vector of its column (dlarfg on rows j+1 ..), so a
// panel needs one launch per column.  Each thread rereads only rows it wrote.
__global__ void __launch_bounds__(1024) k_lr_apply_house(double* __restrict__ Z, int64_t ldz,
                                                         int64_t rows, int64_t j,
                                                         double* __restrict__ tau, int next) {
  __shared__ double red[16];
  __shared__ double sh_alpha, sh_scale;
  const int64_t c = j + 1 + blockIdx.x;
  const double* v = Z + j * ldz;
  double* col = Z + c * ldz;
  if (threadIdx.x == 0) sh_alpha = 0.0;      // (set again below when row c exists)
  const double cj = col[j];                  // read before any thread writes it
  const double tj = tau[j];
  double w = 0.0;
  TIK_LR_ROWS(j + 1, rows, { w += v[r] * col[r]; })
  const double tot = (lr_block_sum<1024>(w, red) + cj) * tj;
  if (threadIdx.x == 0) col[j] = cj - tot;
  const bool head = next && blockIdx.x == 0;
  double ss = 0.0;
  TIK_LR_ROWS(j + 1, rows, {
    const double x = col[r] - tot * v[r];
    col[r] = x;
    if (r == c) sh_alpha = x;
    else ss += x * x;
  })
  if (!head) return;                         // uniform over the block
  const double sigma = lr_block_sum<1024>(ss, red);   // its barriers order sh_alpha
  if (threadIdx.x == 0) lr_house_head(col, c, sh_alpha, sigma, tau, &sh_scale);
  __syncthreads();
  const double sc = sh_scale;
  if (sc != 0.0) TIK_LR_ROWS(c + 1, rows, { col[r] *= sc; })
}
#undef TIK_LR_ROWS

// Explicit panel V (rows k0..rows-1, nb columns, ld rows - k0): unit
// diagonal, zeros above, the stored reflectors below.
__global__ void k_lr_copy_v(const double* __restrict__ Z, int64_t ldz, int64_t rows, int64_t k0,
                            int nb, double* __restrict__ Vc) {
  const int64_t rr = rows - k0;
  const int64_t total = rr * nb;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e % rr, c = e / rr;
    double v;
    if (r < c) v = 0.0;
    else if (r == c) v = 1.0;
    else v = Z[(k0 + r) + (k0 + c) * ldz];
    Vc[e] = v;
  }
}

typedef double lr_qd4 __attribute__((ext_vector_type(4)));

// part[ch] (nb x N, ld nb) = V^T Z over the rows [ch rpc, (ch + 1) rpc) of
// [0, rr): V rr x nb (ld ldv, nb <= 32), Z rr x N (ld ldz).  FP64 MFMA: a
// 32 x 64 output tile per workgroup, one 16-column slice per wave (both
// 16-row halves of V^T), 32-row stages through LDS with the next stage's
// loads in flight.  An empty row range writes zeros.
__global__ void __launch_bounds__(256) k_lr_vtz(int64_t rr, int nb, int64_t N, int64_t rpc,
                                                const double* __restrict__ V, int64_t ldv,
                                                const double* __restrict__ Z, int64_t ldz,
                                                double* __restrict__ part) {
  __shared__ double Vs[32][33];
  __shared__ double Zs[32][65];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t c0 = int64_t(blockIdx.x) * 64;
  const int64_t klo = int64_t(blockIdx.y) * rpc, khi = min(rr, klo + rpc);
  double pv[4], pz[8];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, col = e >> 5, row = e & 31;
      const int64_t k = k0 + row;
      pv[q] = (k < khi && col < nb) ? V[k + col * ldv] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q, col = e >> 5, row = e & 31;
      const int64_t k = k0 + row, j = c0 + col;
      pz[q] = (k < khi && j < N) ? Z[k + j * ldz] : 0.0;
    }
  };
  lr_qd4 acc[2] = {lr_qd4{0, 0, 0, 0}, lr_qd4{0, 0, 0, 0}};
  fetch(klo);
  for (int64_t k0 = klo; k0 < khi; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      Vs[e & 31][e >> 5] = pv[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;
      Zs[e & 31][e >> 5] = pz[q];
    }
    __syncthreads();
    if (k0 + 32 < khi) fetch(k0 + 32);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const double bz = Zs[4 * ks + lk][16 * wv + li];
#pragma unroll
      for (int h = 0; h < 2; ++h)
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[4 * ks + lk][16 * h + li], bz, acc[h], 0, 0, 0);
    }
    __syncthreads();
  }
  double* const out = part + int64_t(blockIdx.y) * nb * N;
  const int64_t j = c0 + 16 * wv + li;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * h + 4 * v + lk;
      if (i < nb && j < N) out[i + j * nb] = acc[h][v];
    }
}

// Z (rr x N, ld ldz) -= V W2 in place: V rr x nb (ld ldv, nb <= 32), W2
// nb x N (ld nb).  FP64 MFMA on W2^T V^T, so that 16 consecutive lanes touch
// 16 consecutive rows of one column of Z: a 128-row x 64-column tile per
// workgroup, 32 rows x 64 columns per wave.
__global__ void __launch_bounds__(256) k_lr_zupd(int64_t rr, int nb, int64_t N,
                                                 const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ W2,
                                                 double* __restrict__ Z, int64_t ldz) {
  __shared__ double Vs[128][33];
  __shared__ double Ws[32][65];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = int64_t(blockIdx.x) * 128, c0 = int64_t(blockIdx.y) * 64;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, col = e >> 7, row = e & 127;
    const int64_t r = r0 + row;
    Vs[row][col] = (r < rr && col < nb) ? V[r + col * ldv] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int e = tid + 256 * q, k = e & 31, col = e >> 5;
    const int64_t jc = c0 + col;
    Ws[k][col] = (k < nb && jc < N) ? W2[k + jc * nb] : 0.0;
  }
  // this wave's tile of Z in the result layout: row li, column 4 v + lk
  double zo[2][4][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 32 * wv + 16 * t + li, col = c0 + 16 * u + 4 * v + lk;
        zo[t][u][v] = (row < rr && col < N) ? Z[row + col * ldz] : 0.0;
      }
  __syncthreads();
  lr_qd4 acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = lr_qd4{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    double vb[2], wa[4];
#pragma unroll
    for (int t = 0; t < 2; ++t) vb[t] = Vs[32 * wv + 16 * t + li][4 * ks + lk];
#pragma unroll
    for (int u = 0; u < 4; ++u) wa[u] = Ws[4 * ks + lk][16 * u + li];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[u], vb[t], acc[t][u], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 32 * wv + 16 * t + li, col = c0 + 16 * u + 4 * v + lk;
        if (row < rr && col < N) Z[row + col * ldz] = zo[t][u][v] - acc[t][u][v];
      }
}

// C = beta C + alpha sum_z part[z] (M x N, ld ldc for both).
__global__ void k_lr_reduce(const double* __restrict__ part, int nz, int64_t M, int64_t N,
                            int64_t ldc, double alpha, double beta, double* __restrict__ C) {
  const int64_t total = M * N;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t mi = e % M, ni = e / M;
    const double* src = part + mi + ni * ldc;
    const int64_t zs = ldc * N;
    // batches of 16 loads in flight, summed in the order z = 0, 1, ...
    double s = 0.0;
    int z = 0;
    for (; z + 16 <= nz; z += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = src[int64_t(z + u) * zs];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; z < nz; ++z) s += src[int64_t(z) * zs];
    const int64_t idx = mi + ni * ldc;
    C[idx] = (beta == 0.0 ? 0.0 : beta * C[idx]) + alpha * s;
  }
}

// T of the compact WY form H_0 ... H_{nb-1} = I - V T V^T from G = V^T V:
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].  One block.
__global__ void k_lr_form_t(const double* __restrict__ G, int nb, const double* __restrict__ tau,
                            double* __restrict__ T) {
  __shared__ double Ts[LR_NB][LR_NB + 1];
  __shared__ double z[LR_NB];
  const int t = threadIdx.x;
  for (int e = t; e < LR_NB * LR_NB; e += blockDim.x) Ts[e % LR_NB][e / LR_NB] = 0.0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t < j) {
      double s = 0.0;
      for (int k = t; k < j; ++k) s += Ts[t][k] * G[k + j * nb];
      z[t] = s;
    }
    __syncthreads();
    if (t < j) Ts[t][j] = -tau[j] * z[t];
    if (t == j) Ts[j][j] = tau[j];
    __syncthreads();
  }
  for (int e = t; e < nb * nb; e += blockDim.x) T[e] = Ts[e % nb][e / nb];
}

// W2 (nb x N) = op(T) W1 with T upper triangular nb x nb; op = transpose when TT.
template <bool TT>
__global__ void k_lr_tmul(const double* __restrict__ T, int nb, const double* __restrict__ W1,
                          int64_t N, double* __restrict__ W2) {
  const int64_t total = int64_t(nb) * N;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e % nb);
    const int64_t c = e / nb;
    double s = 0.0;
    if (TT)
      for (int k = 0; k <= i; ++k) s += T[k + i * nb] * W1[k + c * nb];   // (T^T)[i][k] = T[k][i]
    else
      for (int k = i; k < nb; ++k) s += T[i + k * nb] * W1[k + c * nb];
    W2[e] = s;
  }
}

// ------------------------------------------------- Cholesky QR panels ----
// A panel P (rr x nb, nb <= 32, rr >= nb) of the Householder QR is factored
// in a fixed number of launches instead of one per column: two passes of
// Cholesky QR on the column-scaled Gram matrix give P = Q1 R1, Q1 = Q R2
// with Q orthonormal to rounding when kappa(P D) is moderate (D the column
// scaling), and the compact WY form of a Householder QR with the same
// columns is then rebuilt from Q (the reconstruction of Ballard, Demmel,
// Grigori, Jacquelin, Knight and Nguyen): an LU factorization of the top
// block with the signs S = diag(+-1) chosen on the way, Q_top - S = L W (L
// unit lower, W upper), gives the reflectors V = [L; Q_bot W^{-1}] and
// T = -W S L^{-T}, and then H = I - V T V^T has H^T P = [S R2 R1; 0].
constexpr double LR_CQR_PIVOT = 1e-10;

// R (nb x nb upper, ld nb) with R^T R = G and Rinv = R^{-1}, from the
// Cholesky factor of D G D, D = diag(G)^{-1/2}: R = Rt D^{-1}, R^{-1} = D
// Rt^{-1}.  A pivot of D G D below LR_CQR_PIVOT (or not a number), or a
// diagonal entry of G that is not positive and finite, marks the panel:
// *flag = mark (`first`) or *flag |= mark.  The factors stay finite when the
// panel is marked (pivots are clamped), but are not used.  One thread per
// entry (i, j) = (tid % 32, tid / 32), which keeps its entry in a register;
// each elimination step publishes one row through LDS (two alternating
// buffers, one barrier per step).  (One wavefront holding 16 entries per lane
// measured several times slower: its steps serialize the 16 updates.)
__global__ void __launch_bounds__(1024) k_lr_cqr_chol(const double* __restrict__ G, int nb, int first,
                                                      double* __restrict__ R, double* __restrict__ Rinv,
                                                      int* __restrict__ flag) {
  __shared__ double d[LR_NB];
  __shared__ double rowb[2][LR_NB];
  __shared__ double Rs[LR_NB][LR_NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, i = tid & 31, j = tid >> 5;
  const bool in = i < nb && j < nb;
  if (tid == 0) bad = 0;
  __syncthreads();
  if (tid < nb) {
    const double g = G[tid + tid * nb];
    const bool ok = g > 0.0 && g < INFINITY;
    d[tid] = ok ? 1.0 / sqrt(g) : 1.0;
    if (!ok) bad = 1;
  }
  __syncthreads();
  double a = in ? d[i] * G[i + j * nb] * d[j] : 0.0;
  // D G D = Rt^T Rt (upper): step k publishes row k of the reduced matrix
  for (int k = 0; k < nb; ++k) {
    double* rb = rowb[k & 1];
    if (i == k && j >= k && j < nb) rb[j] = a;
    __syncthreads();
    const double p = rb[k];
    const double pc = p >= LR_CQR_PIVOT ? p : LR_CQR_PIVOT;
    if (tid == 0 && !(p >= LR_CQR_PIVOT)) bad = 1;
    if (i == k && j >= k && j < nb) a = j == k ? sqrt(pc) : a / sqrt(pc);
    else if (i > k && j >= i && j < nb) a -= rb[i] * rb[j] / pc;
  }
  if (in) Rs[i][j] = a;
  __syncthreads();
  // Rt^{-1}, bottom-up and right-looking: step k finishes row k
  double x = i == j ? 1.0 : 0.0;
  for (int k = nb - 1; k >= 0; --k) {
    double* rb = rowb[k & 1];
    if (i == k && j < nb) {
      x = j >= k ? x / Rs[k][k] : 0.0;
      rb[j] = x;
    }
    __syncthreads();
    if (i < k && j < nb) x -= Rs[i][k] * rb[j];
  }
  if (in) {
    R[i + j * nb] = i <= j ? a / d[j] : 0.0;
    Rinv[i + j * nb] = i <= j ? d[i] * x : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    if (first) *flag = bad;
    else if (bad) *flag = 1;
  }
}

// Q[r, :] = P[r, :] B for the rows r0 <= r < rr (B nb x nb upper, ld nb), and
// the same values into Q2 when it is given.  One thread per row, which reads
// its whole row before writing it, so Q may be P (no restrict on them).
__global__ void __launch_bounds__(256) k_lr_cqr_rmul(const double* P, int64_t ldp, int64_t r0, int64_t rr,
                                                     int nb, const double* __restrict__ B, double* Q,
                                                     int64_t ldq, double* Q2, int64_t ldq2) {
  __shared__ double Bs[LR_NB][LR_NB + 1];
  for (int e = threadIdx.x; e < LR_NB * LR_NB; e += 256) {
    const int i = e % LR_NB, j = e / LR_NB;
    Bs[i][j] = (i < nb && j < nb) ? B[i + j * nb] : 0.0;
  }
  __syncthreads();
  const int64_t r = r0 + int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= rr) return;
  double p[LR_NB];
#pragma unroll
  for (int k = 0; k < LR_NB; ++k) p[k] = k < nb ? P[r + k * ldp] : 0.0;
#pragma unroll
  for (int c = 0; c < LR_NB; ++c) {
    if (c < nb) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k <= c; ++k) acc += p[k] * Bs[k][c];
      Q[r + c * ldq] = acc;
      if (Q2) Q2[r + c * ldq2] = acc;
    }
  }
}

// The reconstruction for one panel.  In: the first nb rows of Q1 (rows of
// Vc, ld ldv), R1, R2, R2inv (nb x nb, ld nb).  Out: the panel's top block of
// Zp (ld ldz: S R2 R1 on and above the diagonal, L below it), the top block
// of Vc (L with its unit diagonal, zeros above), T and tau (its diagonal), and
// M = R2^{-1} W^{-1}, which turns the remaining rows of Q1 into the
// reflectors' remaining rows.  One thread per entry (i, j), as in
// k_lr_cqr_chol.
__global__ void __launch_bounds__(1024) k_lr_cqr_recon(double* __restrict__ Vc, int64_t ldv, int nb,
                                                       const double* __restrict__ R1,
                                                       const double* __restrict__ R2,
                                                       const double* __restrict__ R2inv,
                                                       double* __restrict__ Zp, int64_t ldz,
                                                       double* __restrict__ T, double* __restrict__ tau,
                                                       double* __restrict__ M) {
  __shared__ double B1[LR_NB][LR_NB + 1];   // R1
  __shared__ double B2[LR_NB][LR_NB + 1];   // R2
  __shared__ double B2i[LR_NB][LR_NB + 1];  // R2^{-1}
  __shared__ double Qt[LR_NB][LR_NB + 1];   // Q1_top, later L \ W
  __shared__ double Li[LR_NB][LR_NB + 1];   // L^{-1}
  __shared__ double Wi[LR_NB][LR_NB + 1];   // W^{-1}
  __shared__ double rowb[2][LR_NB], colb[2][LR_NB];
  __shared__ double S[LR_NB];
  const int tid = threadIdx.x, i = tid & 31, j = tid >> 5;
  const bool in = i < nb && j < nb;
  if (in) {
    B1[i][j] = R1[i + j * nb];
    B2[i][j] = R2[i + j * nb];
    B2i[i][j] = R2inv[i + j * nb];
    Qt[i][j] = Vc[i + j * ldv];
  }
  __syncthreads();
  // own entry of Q_top = Q1_top R2^{-1}
  double a = 0.0;
  if (in)
    for (int k = 0; k <= j; ++k) a += Qt[i][k] * B2i[k][j];
  // LU without pivoting of Q_top - S, the sign S_p chosen at step p so that
  // the pivot's magnitude is at least 1; step p publishes row p and column p
  for (int p = 0; p < nb; ++p) {
    double* rb = rowb[p & 1];
    double* cb = colb[p & 1];
    if (i == p && j >= p && j < nb) rb[j] = a;
    if (j == p && i > p && i < nb) cb[i] = a;
    __syncthreads();
    const double app = rb[p];
    const double sp = app >= 0.0 ? -1.0 : 1.0;
    const double piv = app - sp;
    if (i == p && j == p) {
      a = piv;
      S[p] = sp;
    } else if (j == p && i > p && i < nb) {
      a = a / piv;
    } else if (i > p && j > p && in) {
      a -= cb[i] / piv * rb[j];
    }
  }
  if (in) Qt[i][j] = a;     // L below the diagonal, W on and above it
  __syncthreads();
  // W^{-1}: bottom-up, right-looking
  double w = i == j ? 1.0 : 0.0;
  for (int k = nb - 1; k >= 0; --k) {
    double* rb = rowb[k & 1];
    if (i == k && j < nb) {
      w = j >= k ? w / Qt[k][k] : 0.0;
      rb[j] = w;
    }
    __syncthreads();
    if (i < k && j < nb) w -= Qt[i][k] * rb[j];
  }
  // L^{-1} (unit diagonal): top-down, right-looking
  double l = i == j ? 1.0 : 0.0;
  for (int k = 0; k < nb; ++k) {
    double* cb = colb[k & 1];
    if (i == k && j < nb) cb[j] = j <= k ? l : 0.0;
    __syncthreads();
    if (i > k && i < nb && j < nb) l -= Qt[i][k] * cb[j];
  }
  if (in) {
    Wi[i][j] = i <= j ? w : 0.0;
    Li[i][j] = i >= j ? l : 0.0;
  }
  __syncthreads();
  if (!in) return;
  // T = -W S L^{-T}, M = R2^{-1} W^{-1}, S R2 R1: entry (i, j), i <= j
  double tv = 0.0, mv = 0.0, rv = 0.0;
  if (i <= j) {
    for (int k = i; k <= j; ++k) {
      tv -= Qt[i][k] * S[k] * Li[j][k];
      mv += B2i[i][k] * Wi[k][j];
      rv += B2[i][k] * B1[k][j];
    }
    rv *= S[i];
  }
  T[i + j * nb] = tv;
  M[i + j * nb] = mv;
  Zp[i + j * ldz] = i <= j ? rv : Qt[i][j];
  Vc[i + j * ldv] = i < j ? 0.0 : (i == j ? 1.0 : Qt[i][j]);
  if (i == j) tau[j] = tv;
}

// 2^-e (up = false) or 2^e (up = true) for the exponent e of the largest
// entry recorded by k_lr_absmax (|e| <= 1000); 1 if it is zero or not finite.
__device__ __forceinline__ double lr_pow2(const unsigned long long* mx, bool up) {
  const double m = __longlong_as_double(static_cast<long long>(*mx));
  if (!(m > 0.0) || !isfinite(m)) return 1.0;
  const int e = min(1000, max(-1000, ilogb(m)));
  return ldexp(1.0, up ? e : -e);
}

// Dst (c x c, ld c) = the transpose of the upper triangle of the factored
// Src (leading c x c block, ld lds): lower triangular, zeros above; times
// lr_pow2(mx, false) when mx is given (an exact power-of-two scaling).
__global__ void k_lr_get_rt(const double* __restrict__ Src, int64_t lds, int64_t c,
                            const unsigned long long* __restrict__ mx, double* __restrict__ Dst) {
  const double sc = mx ? lr_pow2(mx, false) : 1.0;
  const int64_t total = c * c;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % c, j = e / c;            // Dst(i, j) = Src(j, i) sc for j <= i
    Dst[e] = j <= i ? Src[j + i * lds] * sc : 0.0;
  }
}

// Block one-sided Jacobi on the columns of G (s x s, ld s).  Columns in
// blocks of 16; block pairs in round-robin order over nbp = ceil(s / 16)
// rounded up to even (the scalar round-robin schedule, on blocks).  A visit of
// a pair (I, J) replaces the 32 columns C = [C_I C_J] by C Q, Q orthogonal with
// Q^T (C^T C) Q diagonal to the accuracy of one cyclic Jacobi sweep over the
// 32 x 32 Gram matrix.  Each visit is spread over K workgroups, each owning a
// contiguous range of rows_per rows, in two launches per round:
//   k_lr_bgram   partial Gram matrices of the row ranges (FP64 MFMA);
//   k_lr_bapply  their sum in a fixed order, the local Jacobi sweep (the same
//                arithmetic in every workgroup of the pair, so the same Q),
//                then C Q on its row range.
// ver[b] counts the changes of block b; clean[2 (a nbp + b)] holds (ver[a],
// ver[b]) (a < b) from the last visit of the pair that found nothing to
// rotate: a visit with the same versions is skipped (its columns are the ones
// already checked; k_lr_bgram records the decision in flag[pair] for
// k_lr_bapply).  A visit rotating anything adds 1 to *count.  Columns beyond s
// (the last block, the padding block) read as zero and are never written.
typedef double lr_f64x4 __attribute__((ext_vector_type(4)));

struct LrPair {
  int I, J;
  __device__ LrPair(int nbp, int r, int pair) {
    const int m = nbp - 1;
    if (pair == 0) {
      I = r;
      J = m;
    } else {
      I = (r + pair) % m;
      J = ((r - pair) % m + m) % m;
    }
  }
  __device__ int64_t col(int t) const {
    return t < 16 ? int64_t(I) * 16 + t : int64_t(J) * 16 + (t - 16);
  }
};

// Rows [r0, r0 + CH) of the pair's 32 columns (zero at or beyond rhi or s):
// thread tid holds CH / 8 of them, 64 consecutive rows of a column per wave.
template <int CH>
__device__ __forceinline__ void lr_fetch(double (&pf)[CH / 8], const double* __restrict__ G,
                                         int64_t s, const LrPair& P, int64_t r0, int64_t rhi,
                                         int tid) {
#pragma unroll
  for (int q = 0; q < CH / 8; ++q) {
    const int e = tid + 256 * q, col = e / CH, row = e % CH;
    const int64_t c = P.col(col);
    pf[q] = (r0 + row < rhi && c < s) ? G[(r0 + row) + c * s] : 0.0;
  }
}
template <int CH>
__device__ __forceinline__ void lr_stash(double (*T)[33], const double (&pf)[CH / 8], int tid) {
#pragma unroll
  for (int q = 0; q < CH / 8; ++q) {
    const int e = tid + 256 * q;
    T[e % CH][e / CH] = pf[q];
  }
}

__device__ __forceinline__ void lr_pair(int x, int rr, int& p, int& q) {
  if (x == 0) {
    p = rr;
    q = 31;
  } else {
    p = (rr + x) % 31;
    q = (rr - x + 31) % 31;
  }
}

// 1 / x and 1 / sqrt(x) from the hardware estimates and two Newton steps
// each (the estimates carry about half the significand; each step doubles
// it).  For normal x > 0 (lr_rsq) and normal x (lr_rcp).
__device__ __forceinline__ double lr_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double lr_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// Rotation zeroing g_pq of the symmetric 2 x 2 [[gpp, gpq], [gpq, gqq]]
// (new column p = c p - sn q, new column q = sn p + c q), taken when
// |g_pq| > tol sqrt(g_pp g_qq) and |g_pq| > 1e-300: tau = (g_qq - g_pp) /
// (2 g_pq), t the root of t^2 + 2 tau t - 1 = 0 of smaller magnitude,
// c = 1 / sqrt(1 + t^2), sn = t c.  Branch-free: a zero column fails the test
// (0 * inf is NaN), |tau| is clamped at 1e150 (t below 1e-150 either way),
// and whatever the unused arithmetic gives is discarded.  The columns were
// scaled so that the largest entry lies in [1, 2): a column needing the
// 1e-300 floor is negligible against it.
__device__ __forceinline__ bool lr_rot(double gpp, double gqq, double gpq, double tol, double& c,
                                       double& sn) {
  const double agpq = fabs(gpq);
  const bool on = agpq > 1e-300 && agpq * __builtin_amdgcn_rsq(gpp) * __builtin_amdgcn_rsq(gqq) > tol;
  const double tau = (gqq - gpp) * lr_rcp(2.0 * gpq);
  const double at = fmin(fabs(tau), 1e150);
  const double w = 1.0 + at * at;
  const double t = copysign(lr_rcp(at + w * lr_rsq(w)), tau);
  const double cc = lr_rsq(1.0 + t * t);
  c = on ? cc : 1.0;
  sn = on ? t * cc : 0.0;
  return on;
}

template <int CH>
__global__ void __launch_bounds__(256) k_lr_bgram(const double* __restrict__ G, int64_t s, int nbp,
                                                  int r, int K, int64_t rows_per,
                                                  const int* __restrict__ ver,
                                                  const int* __restrict__ clean,
                                                  int* __restrict__ flag, double* __restrict__ part) {
  static_assert(CH % 128 == 0, "chunk rows: a multiple of 128");
  __shared__ double T[CH][33];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pair = blockIdx.x / K, k = blockIdx.x % K;
  const LrPair P(nbp, r, pair);
  const int ba = min(P.I, P.J), bb = max(P.I, P.J);
  const int* const cl = clean + 2 * (int64_t(ba) * nbp + bb);
  const bool skip = cl[0] == ver[ba] && cl[1] == ver[bb];
  if (k == 0 && tid == 0) flag[pair] = skip ? 1 : 0;
  if (skip) return;                          // uniform
  const int64_t rlo = int64_t(k) * rows_per, rhi = min(s, rlo + rows_per);
  // one 16 x 16 tile of C^T C per wave; four accumulator chains, operands
  // read from LDS eight steps at a time
  const int wr = 16 * (wv & 1), wc = 16 * (wv >> 1);
  lr_f64x4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = lr_f64x4{0, 0, 0, 0};
  double pf[CH / 8];
  lr_fetch<CH>(pf, G, s, P, rlo, rhi, tid);
  for (int64_t r0 = rlo; r0 < rhi; r0 += CH) {
    lr_stash<CH>(T, pf, tid);
    __syncthreads();
    if (r0 + CH < rhi) lr_fetch<CH>(pf, G, s, P, r0 + CH, rhi, tid);
    for (int kb = 0; kb < CH / 4; kb += 8) {
      double x[8], y[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        x[j] = T[4 * (kb + j) + lk][wr + li];
        y[j] = T[4 * (kb + j) + lk][wc + li];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        acc[j & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[j], y[j], acc[j & 3], 0, 0, 0);
    }
    __syncthreads();
  }
  double* const out = part + (int64_t(pair) * K + k) * 1024;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    out[(wr + 4 * v + lk) * 32 + wc + li] = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
}

template <int CH>
__global__ void __launch_bounds__(256) k_lr_bapply(double* __restrict__ G, int64_t s, int nbp, int r,
                                                   int K, int64_t rows_per, double tol,
                                                   int* __restrict__ ver, int* __restrict__ clean,
                                                   const int* __restrict__ flag,
                                                   const double* __restrict__ part,
                                                   unsigned int* __restrict__ count) {
  static_assert(CH % 128 == 0, "chunk rows: a multiple of 128");
  __shared__ double T[CH][33];
  __shared__ double Gs[2][32][33];
  __shared__ double Qs[32][33];
  __shared__ int rot;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pair = blockIdx.x / K, k = blockIdx.x % K;
  if (flag[pair]) return;                    // uniform
  const LrPair P(nbp, r, pair);
  // 1. the Gram matrix: partial sums in a fixed order
  const double* const pp = part + int64_t(pair) * K * 1024;
  {
    // every partial this thread needs is loaded before the sums (up to 16 in
    // flight); the sums keep the order k = 0, 1, ...
    double g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) g[q] = pp[tid + 256 * q];
    for (int k0 = 1; k0 < K; k0 += 4) {
      double v[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[u][q] = k0 + u < K ? pp[int64_t(k0 + u) * 1024 + tid + 256 * q] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k0 + u < K) g[q] += v[u][q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      Gs[0][e >> 5][e & 31] = g[q];
      Qs[e >> 5][e & 31] = (e >> 5) == (e & 31) ? 1.0 : 0.0;
    }
  }
  if (tid == 0) rot = 0;
  __syncthreads();
  // 2. one cyclic Jacobi sweep on it: G <- J^T G J, Q <- Q J.  Each round
  // rotates 16 disjoint pairs; thread (xa, xb) forms the 2 x 2 block of the
  // pairs xa (rows) and xb (columns) from the previous round's copy, and
  // rotates columns (pb, qb) of Q in rows 2 xa, 2 xa + 1.  Every thread forms
  // the two rotations it needs itself: forming each once, in 16 threads, costs
  // a second barrier per round and measured slower (the rounds are bound by the
  // rotation's chain of dependent operations, not by its arithmetic).
  const int xa = tid >> 4, xb = tid & 15;
  int cur = 0;
  for (int rr = 0; rr < 31; ++rr) {
    int pa, qa, pb, qb;
    lr_pair(xa, rr, pa, qa);
    lr_pair(xb, rr, pb, qb);
    const double(*g)[33] = Gs[cur];
    const double apa = g[pa][pa], aqa = g[qa][qa], ao = g[pa][qa];
    const double bpb = g[pb][pb], bqb = g[qb][qb], bo = g[pb][qb];
    const double g1 = g[pa][pb], g2 = g[pa][qb], g3 = g[qa][pb], g4 = g[qa][qb];
    const double q1 = Qs[2 * xa][pb], q2 = Qs[2 * xa][qb];
    const double q3 = Qs[2 * xa + 1][pb], q4 = Qs[2 * xa + 1][qb];
    double ca, sa, cb, sb;
    const bool on_a = lr_rot(apa, aqa, ao, tol, ca, sa);
    lr_rot(bpb, bqb, bo, tol, cb, sb);
    const double xpp = cb * g1 - sb * g2, xpq = sb * g1 + cb * g2;
    const double xqp = cb * g3 - sb * g4, xqq = sb * g3 + cb * g4;
    double(*h)[33] = Gs[cur ^ 1];
    h[pa][pb] = ca * xpp - sa * xqp;
    h[qa][pb] = sa * xpp + ca * xqp;
    h[pa][qb] = ca * xpq - sa * xqq;
    h[qa][qb] = sa * xpq + ca * xqq;
    Qs[2 * xa][pb] = cb * q1 - sb * q2;
    Qs[2 * xa][qb] = sb * q1 + cb * q2;
    Qs[2 * xa + 1][pb] = cb * q3 - sb * q4;
    Qs[2 * xa + 1][qb] = sb * q3 + cb * q4;
    if (on_a && xb == 0) rot = 1;
    cur ^= 1;
    __syncthreads();
  }
  if (!rot) {                                // uniform: read after the barrier above
    if (k == 0 && tid == 0) {
      const int ba = min(P.I, P.J), bb = max(P.I, P.J);
      int* const cl = clean + 2 * (int64_t(ba) * nbp + bb);
      cl[0] = ver[ba];
      cl[1] = ver[bb];
    }
    return;
  }
  // 3. C <- C Q on this workgroup's rows, computed transposed (Q^T C^T) so
  // that 16 consecutive lanes store 16 consecutive rows of one column
  const int64_t rlo = int64_t(k) * rows_per, rhi = min(s, rlo + rows_per);
  const int oc = 16 * (wv & 1), rh = (CH / 2) * (wv >> 1);
  double qv[8];                              // this wave's Q^T operand, all 8 steps
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) qv[ks] = Qs[4 * ks + lk][oc + li];
  double pf[CH / 8];
  lr_fetch<CH>(pf, G, s, P, rlo, rhi, tid);
  for (int64_t r0 = rlo; r0 < rhi; r0 += CH) {
    lr_stash<CH>(T, pf, tid);
    __syncthreads();
    if (r0 + CH < rhi) lr_fetch<CH>(pf, G, s, P, r0 + CH, rhi, tid);
    // four row tiles at a time: four independent accumulator chains
#pragma unroll
    for (int rt = 0; rt < CH / 32; rt += 4) {
      lr_f64x4 o[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) o[u] = lr_f64x4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        double y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = T[rh + 16 * (rt + u) + li][4 * ks + lk];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          o[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv[ks], y[u], o[u], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t row = r0 + rh + 16 * (rt + u) + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t c = P.col(oc + 4 * v + lk);
          if (row < rhi && c < s) G[row + c * s] = o[u][v];
        }
      }
    }
    __syncthreads();
  }
  if (k == 0 && tid == 0) {
    ver[P.I] += 1;
    ver[P.J] += 1;
    atomicAdd(count, 1u);
  }
}

// Largest |Src(j, i)|, j <= i (the upper triangle of Src, c x c, ld lds), as
// the bit pattern of a non-negative double, into *mx (which starts at 0).
__global__ void __launch_bounds__(256) k_lr_absmax(const double* __restrict__ Src, int64_t lds,
                                                   int64_t c, unsigned long long* __restrict__ mx) {
  __shared__ double red[4];
  double m = 0.0;
  const int64_t total = c * c;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
    const int64_t i = e % c, j = e / c;
    if (j <= i) m = fmax(m, fabs(Src[j + i * lds]));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(mx, static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}


// sigma_j = ||g_j||, g_j /= sigma_j (one block per column).
__global__ void __launch_bounds__(256) k_lr_normalize(double* __restrict__ G, int64_t s,
                                                      const unsigned long long* __restrict__ mx,
                                                      double* __restrict__ sig) {
  __shared__ double red[4];
  double* g = G + int64_t(blockIdx.x) * s;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < s; i += 256) ss += g[i] * g[i];
  const double nrm = sqrt(lr_block_sum<256>(ss, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = threadIdx.x; i < s; i += 256) g[i] *= inv;
  if (threadIdx.x == 0) sig[blockIdx.x] = nrm * lr_pow2(mx, true);
}

// Descending order of sigma (bitonic sort of (sigma, index) in LDS, s <= 4096);
// Zs[:, k] = G[:, perm[k]] padded with n - s zero rows (X = [Z; 0], n x s).
__global__ void __launch_bounds__(1024) k_lr_sort(const double* __restrict__ sig, int64_t s,
                                                  int32_t* __restrict__ perm,
                                                  double* __restrict__ sig_sorted) {
  __shared__ double key[4096];
  __shared__ int32_t idx[4096];
  int P = 1;
  while (P < s) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    key[i] = i < s ? sig[i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  for (int len = 2; len <= P; len <<= 1) {
    for (int str = len >> 1; str > 0; str >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int j = i ^ str;
        if (j > i) {
          const bool desc = (i & len) == 0;
          const double a = key[i], b = key[j];
          const bool swap = desc ? (a < b || (a == b && idx[i] > idx[j]))
                                 : (a > b || (a == b && idx[i] < idx[j]));
          if (swap) {
            key[i] = b;
            key[j] = a;
            const int32_t t = idx[i];
            idx[i] = idx[j];
            idx[j] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < s; i += blockDim.x) {
    perm[i] = idx[i];
    sig_sorted[i] = key[i];
  }
}

__global__ void k_lr_gather(const double* __restrict__ G, int64_t s, int64_t n,
                            const int32_t* __restrict__ perm, double* __restrict__ X) {
  const int64_t total = n * s;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    X[e] = r < s ? G[r + int64_t(perm[c]) * s] : 0.0;
  }
}

// S_i[j] = 1 - (1 + sigma_j^2 / lam_i)^(-1/2) for j < s_i, else 0 (Algorithm 3 step 7).
__global__ void k_lr_S(const double* __restrict__ sig, int64_t s, const double* __restrict__ lams,
                       const int32_t* __restrict__ si, int N, double* __restrict__ S) {
  const int64_t total = int64_t(N) * s;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e / s);
    const int64_t j = e % s;
    const double sg = sig[j];
    S[e] = j < si[i] ? 1.0 - 1.0 / sqrt(1.0 + sg * sg / lams[i]) : 0.0;
  }
}

// ------------------------------------------------------------- host side ----
static unsigned lr_grid(int64_t total) {
  return unsigned(std::min<int64_t>(std::max<int64_t>(cdiv(total, 256), 1), 8192));
}

// op(A) B for the QR updates, split over K into nz slices of `part`.
// W (nb x N, ld nb) = V^T Z (V rr x nb, Z rr x N): row chunks on about 512
// workgroups in all, partial products reduced in a fixed order.
static int lr_vtz(int64_t rr, int nb, int64_t N, const double* V, int64_t ldv, const double* Z,
                  int64_t ldz, double* W, double* part, int64_t part_cap, hipStream_t st) {
  const int64_t ct = cdiv(N, 64);
  int64_t nch = std::max<int64_t>(1, std::min<int64_t>(cdiv(512, ct), cdiv(rr, 128)));
  while (nch > 1 && nch * nb * N > part_cap) --nch;
  const int64_t rpc = cdiv(cdiv(rr, nch), 32) * 32;
  nch = std::max<int64_t>(1, cdiv(rr, rpc));
  hipLaunchKernelGGL(k_lr_vtz, dim3(unsigned(ct), unsigned(nch)), dim3(256), 0, st, rr, nb, N, rpc, V,
                     ldv, Z, ldz, part);
  TIK_LAUNCHED("k_lr_vtz");
  hipLaunchKernelGGL(k_lr_reduce, dim3(lr_grid(int64_t(nb) * N)), dim3(256), 0, st, part, int(nch),
                     int64_t(nb), N, int64_t(nb), 1.0, 0.0, W);
  TIK_LAUNCHED("k_lr_reduce");
  return TIK_OK;
}
// Z (rr x N, ld ldz) -= V W2 (V rr x nb, W2 nb x N).
static int lr_zupd(int64_t rr, int nb, int64_t N, const double* V, int64_t ldv, const double* W2,
                   double* Z, int64_t ldz, hipStream_t st) {
  hipLaunchKernelGGL(k_lr_zupd, dim3(unsigned(cdiv(rr, 128)), unsigned(cdiv(N, 64))), dim3(256), 0, st,
                     rr, nb, N, V, ldv, W2, Z, ldz);
  TIK_LAUNCHED("k_lr_zupd");
  return TIK_OK;
}

struct QrWs {
  double* tau;    // cols
  double* T;      // ceil(cols / 32) panels of 32 x 32
  double* Vc;     // rows x 32
  double* Gm;     // 32 x 32
  double* W1;     // 32 x cols
  double* W2;     // 32 x cols
  double* part;   // part_cap
  int64_t part_cap;
  double *R1, *R1i, *R2, *R2i, *M;   // 32 x 32 each: the Cholesky QR panel factors
  int* flag;                         // the panel's Cholesky QR mark
};

static size_t qr_ws_doubles(int64_t rows, int64_t cols) {
  const int64_t np = cdiv(cols, LR_NB);
  return size_t(cols + np * LR_NB * LR_NB + rows * LR_NB + LR_NB * LR_NB + 2 * LR_NB * cols +
                64 * LR_NB * std::max<int64_t>(cols, LR_NB) + 5 * LR_NB * LR_NB + 8 + 8 * 32);
}

static QrWs qr_ws_carve(double* base, int64_t rows, int64_t cols) {
  QrWs w;
  const int64_t np = cdiv(cols, LR_NB);
  w.tau = base;
  w.T = w.tau + cols;
  w.Vc = w.T + np * LR_NB * LR_NB;
  w.Gm = w.Vc + rows * LR_NB;
  w.W1 = w.Gm + LR_NB * LR_NB;
  w.W2 = w.W1 + LR_NB * cols;
  w.part = w.W2 + LR_NB * cols;
  w.part_cap = 64 * LR_NB * std::max<int64_t>(cols, LR_NB);
  w.R1 = w.part + w.part_cap;
  w.R1i = w.R1 + LR_NB * LR_NB;
  w.R2 = w.R1i + LR_NB * LR_NB;
  w.R2i = w.R2 + LR_NB * LR_NB;
  w.M = w.R2i + LR_NB * LR_NB;
  w.flag = reinterpret_cast<int*>(w.M + LR_NB * LR_NB);
  return w;
}

// In-place Householder QR of Z (rows x cols, ld ldz, rows >= cols): R in the
// upper triangle, reflectors below it, tau and the per-panel T factors of the
// compact WY form H_k0 ... H_k0+nb-1 = I - V T V^T in w.
static int qr_factor(double* Z, int64_t rows, int64_t cols, int64_t ldz, const QrWs& w,
                     hipStream_t st) {
  const int64_t np = cdiv(cols, LR_NB);
  for (int64_t pnl = 0; pnl < np; ++pnl) {
    const int64_t k0 = pnl * LR_NB;
    const int nb = int(std::min<int64_t>(LR_NB, cols - k0));
    const int64_t rr = rows - k0;
    double* const P = Z + k0 + k0 * ldz;
    double* Tp = w.T + pnl * LR_NB * LR_NB;
    bool cqr = false;
    if (option_cholqr_panels()) {
      // two Cholesky QR passes; the host reads the panel's mark before anything
      // in Z is written, so a marked panel is still intact for the fallback
      ProfScope ps_c("lr_cqr", st);
      TIK_TRY(lr_vtz(rr, nb, nb, P, ldz, P, ldz, w.Gm, w.part, w.part_cap, st));
      hipLaunchKernelGGL(k_lr_cqr_chol, dim3(1), dim3(1024), 0, st, w.Gm, nb, 1, w.R1, w.R1i, w.flag);
      TIK_LAUNCHED("k_lr_cqr_chol");
      hipLaunchKernelGGL(k_lr_cqr_rmul, dim3(unsigned(cdiv(rr, 256))), dim3(256), 0, st, P, ldz, int64_t(0),
                         rr, nb, w.R1i, w.Vc, rr, static_cast<double*>(nullptr), int64_t(0));
      TIK_LAUNCHED("k_lr_cqr_rmul");
      TIK_TRY(lr_vtz(rr, nb, nb, w.Vc, rr, w.Vc, rr, w.Gm, w.part, w.part_cap, st));
      hipLaunchKernelGGL(k_lr_cqr_chol, dim3(1), dim3(1024), 0, st, w.Gm, nb, 0, w.R2, w.R2i, w.flag);
      TIK_LAUNCHED("k_lr_cqr_chol");
      int mark = 1;
      TIK_HIP(hipMemcpyAsync(&mark, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
      TIK_HIP(hipStreamSynchronize(st));
      if (mark == 0) {
        ProfScope ps_r("lr_cqr_recon", st);
        hipLaunchKernelGGL(k_lr_cqr_recon, dim3(1), dim3(1024), 0, st, w.Vc, rr, nb, w.R1, w.R2, w.R2i, P, ldz,
                           Tp, w.tau + k0, w.M);
        TIK_LAUNCHED("k_lr_cqr_recon");
        if (rr > nb) {
          hipLaunchKernelGGL(k_lr_cqr_rmul, dim3(unsigned(cdiv(rr - nb, 256))), dim3(256), 0, st, w.Vc, rr,
                             int64_t(nb), rr, nb, w.M, w.Vc, rr, P, ldz);
          TIK_LAUNCHED("k_lr_cqr_rmul");
        }
        cqr = true;
      }
    }
    if (!cqr) {
      ProfScope ps_h("lr_colqr", st);
      // reflector of the panel's first column, then per column one launch that
      // applies H_j to the rest of the panel and forms the reflector of j + 1
      hipLaunchKernelGGL(k_lr_house, dim3(1), dim3(1024), 0, st, Z, ldz, rows, k0, w.tau);
      TIK_LAUNCHED("k_lr_house");
      for (int jj = 0; jj + 1 < nb; ++jj)
        hipLaunchKernelGGL(k_lr_apply_house, dim3(unsigned(nb - jj - 1)), dim3(1024), 0, st, Z, ldz,
                           rows, k0 + jj, w.tau, 1);
      TIK_LAUNCHED("k_lr_apply_house");
      hipLaunchKernelGGL(k_lr_copy_v, dim3(lr_grid(rr * nb)), dim3(256), 0, st, Z, ldz, rows, k0, nb,
                         w.Vc);
      TIK_LAUNCHED("k_lr_copy_v");
      TIK_TRY(lr_vtz(rr, nb, nb, w.Vc, rr, w.Vc, rr, w.Gm, w.part, w.part_cap, st));
      hipLaunchKernelGGL(k_lr_form_t, dim3(1), dim3(64), 0, st, w.Gm, nb, w.tau + k0, Tp);
      TIK_LAUNCHED("k_lr_form_t");
    }
    const int64_t ntr = cols - k0 - nb;
    if (ntr > 0) {
      ProfScope ps_t("lr_trail", st);
      double* Ztr = Z + k0 + (k0 + nb) * ldz;
      // W1 = Vc^T Ztr (nb x ntr), W2 = T^T W1, Ztr -= Vc W2
      TIK_TRY(lr_vtz(rr, nb, ntr, w.Vc, rr, Ztr, ldz, w.W1, w.part, w.part_cap, st));
      hipLaunchKernelGGL(k_lr_tmul<true>, dim3(lr_grid(nb * ntr)), dim3(256), 0, st, Tp, nb, w.W1,
                         ntr, w.W2);
      TIK_LAUNCHED("k_lr_tmul");
      TIK_TRY(lr_zupd(rr, nb, ntr, w.Vc, rr, w.W2, Ztr, ldz, st));
    }
  }
  return TIK_OK;
}

// X (rows x c, ld ldx) <- Q X with Q the product of the reflectors stored in
// Z by qr_factor (applied last panel first).
static int qr_apply_q(const double* Z, int64_t rows, int64_t cols, int64_t ldz, const QrWs& w,
                      double* X, int64_t c, int64_t ldx, hipStream_t st) {
  const int64_t np = cdiv(cols, LR_NB);
  for (int64_t pnl = np - 1; pnl >= 0; --pnl) {
    const int64_t k0 = pnl * LR_NB;
    const int nb = int(std::min<int64_t>(LR_NB, cols - k0));
    const int64_t rr = rows - k0;
    hipLaunchKernelGGL(k_lr_copy_v, dim3(lr_grid(rr * nb)), dim3(256), 0, st, Z, ldz, rows, k0, nb,
                       w.Vc);
    TIK_LAUNCHED("k_lr_copy_v");
    double* Xr = X + k0;
    TIK_TRY(lr_vtz(rr, nb, c, w.Vc, rr, Xr, ldx, w.W1, w.part, w.part_cap, st));
    hipLaunchKernelGGL(k_lr_tmul<false>, dim3(lr_grid(nb * c)), dim3(256), 0, st,
                       w.T + pnl * LR_NB * LR_NB, nb, w.W1, c, w.W2);
    TIK_LAUNCHED("k_lr_tmul");
    TIK_TRY(lr_zupd(rr, nb, c, w.Vc, rr, w.W2, Xr, ldx, st));
  }
  return TIK_OK;
}

// ------------------------------------------------------ BP2 fallback -------
// Z ((s + k) x k, ld s + k) = [Y; sqrt(lam) I_k], Y s x k (ld s).
__global__ void k_bp2_stack(const double* __restrict__ Y, int64_t s, int64_t k, double sq,
                            double* __restrict__ Z) {
  const int64_t rows = s + k;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < rows * k;
       e += int64_t(gridDim.x) * 256) {
    const int64_t r = e % rows, c = e / rows;
    Z[e] = r < s ? Y[r + c * s] : (r - s == c ? sq : 0.0);
  }
}

// R (k x k, ld k) = the upper triangle of Z's leading k x k block, zeros below.
__global__ void k_bp2_take_r(const double* __restrict__ Z, int64_t ldz, int64_t k,
                             double* __restrict__ R) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < k * k; e += int64_t(gridDim.x) * 256) {
    const int64_t r = e % k, c = e / k;
    R[e] = r <= c ? Z[r + c * ldz] : 0.0;
  }
}

size_t bp2_scratch_doubles(int64_t s, int64_t k) {
  return size_t((s + k) * k) + qr_ws_doubles(s + k, k) + 64;
}

// R with R^T R = Y^T Y + lam I from the Householder QR of [Y; sqrt(lam) I]
// (the BP2 preconditioner of Section 4.1; R's diagonal may carry either sign,
// which R^{-1} absorbs).  The Gram matrix is never formed, so the factor
// exists however ill-conditioned Y^T Y + lam I is.
int launch_bp2_r(const double* Y, int64_t s, int64_t k, double lam, double* R, double* scratch,
                 hipStream_t st) {
  ProfScope ps("bp2", st);
  const int64_t rows = s + k;
  double* Z = scratch;
  const QrWs w = qr_ws_carve(Z + rows * k, rows, k);
  hipLaunchKernelGGL(k_bp2_stack, dim3(lr_grid(rows * k)), dim3(256), 0, st, Y, s, k, std::sqrt(lam), Z);
  TIK_LAUNCHED("k_bp2_stack");
  TIK_TRY(qr_factor(Z, rows, k, rows, w, st));
  hipLaunchKernelGGL(k_bp2_take_r, dim3(lr_grid(k * k)), dim3(256), 0, st, Z, rows, k, R);
  TIK_LAUNCHED("k_bp2_take_r");
  return TIK_OK;
}

// Block Jacobi bookkeeping, in doubles: the scaling maximum (1), the partial
// Gram matrices (npairs K <= kLrWg of them, 1024 each), then ints: ver (nbp),
// clean (2 nbp^2) and flag (nbp / 2).
// About kLrWg workgroups per round in all: K = kLrWg / (s / 32) per visit.
// At s = 1844 (58 pairs) K = 4 measured fastest: the sweeps took 99, 70, 51,
// 63 and 101 ms with K = 1, 2, 4, 8 and 15 (fewer rows per workgroup, but
// every workgroup repeats the visit's 32 x 32 sweep and more of them share a
// compute unit).
constexpr int kLrWg = 256;
static int64_t lr_nbp(int64_t s) {
  const int64_t nblk = cdiv(s, 16);
  return nblk + (nblk & 1);
}
static size_t lr_book_doubles(int64_t s) {
  const int64_t nbp = lr_nbp(s);
  return size_t(1 + int64_t(kLrWg) * 1024 + cdiv(nbp + 2 * nbp * nbp + nbp / 2, 2));
}

size_t lowrank_scratch_doubles(int64_t n, int64_t s) {
  // Z (n s) + Z2 (s s) + L (s s) + sig_raw (s) + QR workspaces of n x s and
  // s x s + the block Jacobi bookkeeping
  return size_t(n * s + 2 * s * s + s) + qr_ws_doubles(n, s) + qr_ws_doubles(s, s) +
         lr_book_doubles(s) + 64;
}

// V (n x s, ld n, columns by decreasing sigma) and sigma (s) of Y (s x n, ld s).
// `scratch` holds lowrank_scratch_doubles(n, s) doubles; `cnt` one counter.
int launch_lowrank_svd(const double* Y, int64_t s, int64_t n, double* V, double* sig,
                       double* scratch, unsigned int* cnt, int32_t* perm, int* sweeps_out,
                       hipStream_t st) {
  ProfScope ps("lowrank", st);
  if (s > 4096) {
    set_error("internal: low-rank SVD supports s <= 4096");
    return TIK_EINVAL;
  }
  double* Z = scratch;               // n x s: Y^T, then R1 and the reflectors of Q1
  double* Z2 = Z + n * s;            // s x s: R1^T, then R2 and the reflectors of Q2
  double* L = Z2 + s * s;            // s x s: R2^T, rotated into Z Sigma
  double* sig_raw = L + s * s;       // s
  const QrWs w1 = qr_ws_carve(sig_raw + s, n, s);
  const QrWs w2 = qr_ws_carve(sig_raw + s + qr_ws_doubles(n, s), s, s);
  double* const book = sig_raw + s + qr_ws_doubles(n, s) + qr_ws_doubles(s, s);
  unsigned long long* const mx = reinterpret_cast<unsigned long long*>(book);
  double* const part = book + 1;
  int* const ver = reinterpret_cast<int*>(part + int64_t(kLrWg) * 1024);
  {
    ProfScope ps_qr("lr_qr", st);
    // 1. Y^T = Q1 R1
    hipLaunchKernelGGL(k_lr_transpose, dim3(unsigned(cdiv(s, 32)), unsigned(cdiv(n, 32))), dim3(256),
                       0, st, Y, s, n, Z);
    TIK_LAUNCHED("k_lr_transpose");
    TIK_TRY(qr_factor(Z, n, s, n, w1, st));
    // 2. R1^T = Q2 R2, L = R2^T
    hipLaunchKernelGGL(k_lr_get_rt, dim3(lr_grid(s * s)), dim3(256), 0, st, Z, n, s,
                       static_cast<const unsigned long long*>(nullptr), Z2);
    TIK_LAUNCHED("k_lr_get_rt");
    TIK_TRY(qr_factor(Z2, s, s, s, w2, st));
    // L = R2^T scaled by a power of two so that its largest entry lies in
    // [1, 2): the Gram entries of the rotations stay clear of under- and
    // overflow whatever the scale of A; sigma is scaled back exactly
    TIK_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_lr_absmax, dim3(lr_grid(s * s)), dim3(256), 0, st, Z2, s, s, mx);
    TIK_LAUNCHED("k_lr_absmax");
    hipLaunchKernelGGL(k_lr_get_rt, dim3(lr_grid(s * s)), dim3(256), 0, st, Z2, s, s,
                       static_cast<const unsigned long long*>(mx), L);
    TIK_LAUNCHED("k_lr_get_rt");
  }
  // 3. one-sided Jacobi on the columns of L
  const double tol = 1e-15 * std::sqrt(double(s));
  int sweeps = 0;
  const int maxsweeps = 30;
  const int nbp = int(lr_nbp(s)), npairs = nbp / 2;
  // workgroups per visit: about kLrWg in all, at least 128 rows each
  const int K = std::max(1, std::min(kLrWg / npairs, int(cdiv(s, 128))));
  const int64_t rows_per = cdiv(cdiv(s, K), 32) * 32;
  int* const clean = ver + nbp;
  int* const flag = clean + 2 * nbp * nbp;
  TIK_HIP(hipMemsetAsync(ver, 0, sizeof(int) * size_t(nbp), st));
  TIK_HIP(hipMemsetAsync(clean, 0xff, sizeof(int) * 2 * size_t(nbp) * size_t(nbp), st));
  const dim3 grid(unsigned(npairs * K));
  for (; sweeps < maxsweeps;) {
    ProfScope ps_sw("lr_sweep", st);
    TIK_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned int), st));
    for (int r = 0; r < nbp - 1; ++r) {
      hipLaunchKernelGGL(k_lr_bgram<128>, grid, dim3(256), 0, st, L, s, nbp, r, K, rows_per, ver,
                         clean, flag, part);
      hipLaunchKernelGGL(k_lr_bapply<128>, grid, dim3(256), 0, st, L, s, nbp, r, K, rows_per, tol, ver,
                         clean, flag, part, cnt);
    }
    TIK_LAUNCHED("k_lr_bapply");
    ++sweeps;
    unsigned int h = 0;
    TIK_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    TIK_HIP(hipStreamSynchronize(st));
    if (h == 0) break;
  }
  if (sweeps_out) *sweeps_out = sweeps;
  hipLaunchKernelGGL(k_lr_normalize, dim3(unsigned(s)), dim3(256), 0, st, L, s,
                     static_cast<const unsigned long long*>(mx), sig_raw);
  TIK_LAUNCHED("k_lr_normalize");
  hipLaunchKernelGGL(k_lr_sort, dim3(1), dim3(1024), 0, st, sig_raw, s, perm, sig);
  TIK_LAUNCHED("k_lr_sort");
  // 4. V = Q1 [Z; 0]
  ProfScope ps_q("lr_q", st);
  hipLaunchKernelGGL(k_lr_gather, dim3(lr_grid(n * s)), dim3(256), 0, st, L, s, n, perm, V);
  TIK_LAUNCHED("k_lr_gather");
  return qr_apply_q(Z, n, s, n, w1, V, s, n, st);
}

int launch_lowrank_S(const double* sig, int64_t s, const double* lams, const int32_t* si, int N,
                     double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_lr_S, dim3(lr_grid(int64_t(N) * s)), dim3(256), 0, st, sig, s, lams, si, N, S);
  TIK_LAUNCHED("k_lr_S");
  return TIK_OK;
}


// ===================================================== low-rank apply =======
// R_i^{-1} x = lam_i^{-1/2} (x - V S_i V^T x) (eq. RinvOver, Algorithm 3 step 8)
// for all lambdas of a solve at once; the matrix is symmetric, so the same
// three kernels give R^{-T}.  V (k x s, ld k) is read twice per application:
//   proj    part[ch][j][i] = sum_{r in chunk ch} V[r, j] x_i[r]     (j < smax)
//   coef    c[j, i] = S_i[j] sum_ch part[ch][j][i]
//   expand  opart[jc][i][r] = sum_{j in column chunk jc} V[r, j] c[j, i]
//   fin     the LSQR step that consumes R^{-1} x, with the chunk sums of opart.
// S_i[j] is zero for j >= s_i, which truncates every lambda to its own rank.

// K values per lane reduced over the 64 lanes: halving exchanges (K/2 + K/4
// + ... shuffles) leave lane l with the total of value l >> (6 - log2 K).
template <int K>
__device__ __forceinline__ void lr_xreduce(double (&v)[K], int lane) {
  int h = K;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    if (h > 1) {
      h >>= 1;
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int q = 0; q < K / 2; ++q) {
        if (q < h) {
          const double send = up ? v[q] : v[q + h];
          const double keep = up ? v[q + h] : v[q];
          v[q] = keep + __shfl_xor(send, o, 64);
        }
      }
    } else {
      v[0] += __shfl_xor(v[0], o, 64);
    }
  }
}

template <int NC, int CPW, bool LMAJ>
__global__ void __launch_bounds__(256) k_lr_proj(const DevProb* __restrict__ P,
                                                 const Item* __restrict__ items, int N,
                                                 const double* __restrict__ src,
                                                 double* __restrict__ part) {
  constexpr int K = CPW * NC;
  static_assert(K <= 64, "values per lane");
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t k = pr.k;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j0 = int64_t(it.blk) * (4 * CPW) + int64_t(wv) * CPW;
  const int64_t rb = int64_t(it.ch) * pr.lrRch, re = min(k, rb + pr.lrRch);
  const double* __restrict__ V = pr.V;
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (int64_t r = rb + lane; r < re; r += 64) {
    double xv[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i)
      xv[i] = i < N ? (LMAJ ? src[pr.offS * N + int64_t(i) * k + r] : src[(pr.offS + r) * N + i]) : 0.0;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const double vq = (j0 + q < pr.smax) ? V[r + (j0 + q) * k] : 0.0;
#pragma unroll
      for (int i = 0; i < NC; ++i) acc[q * NC + i] = fma(vq, xv[i], acc[q * NC + i]);
    }
  }
  lr_xreduce<K>(acc, lane);
  constexpr int G = 64 / K;
  if ((lane & (G - 1)) == 0) {
    const int idx = lane / G, q = idx / NC, i = idx % NC;
    const int64_t j = j0 + q;
    if (j < pr.smax && i < N) part[pr.lrPart + (int64_t(it.ch) * pr.s + j) * N + i] = acc[0];
  }
}

// Projection on the matrix cores (16 or 32 lambdas): block = 128 columns of V
// x one row chunk; wave w owns columns 32 w .. 32 w + 31, as two 16-column
// tiles times NC / 16 lambda tiles of v_mfma_f64_16x16x4_f64.  V (32 rows x
// 128 columns) and x (32 rows x NC) are staged through LDS, the next tile
// being fetched into registers while the current one is consumed.  Blocks are
// remapped so that the column blocks of one row chunk, which share x, run on
// one XCD.
typedef double lr_d4 __attribute__((ext_vector_type(4)));

template <int NC, bool LMAJ>
__global__ void __launch_bounds__(256) k_lr_proj_mfma(const DevProb* __restrict__ P,
                                                      const Item* __restrict__ items, int nitems,
                                                      int N, const double* __restrict__ src,
                                                      double* __restrict__ part) {
  constexpr int NT = NC / 16;
  constexpr int CB = 128, RS = 32, AP = RS + 2, UP = NC + 1;
  __shared__ double Vs[CB][AP];
  __shared__ double Xs[RS][UP];
  const int g = blockIdx.x;
  const int per = (nitems + 7) >> 3;
  const int L = (g & 7) * per + (g >> 3);
  if (L >= nitems) return;
  const Item it = items[L];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const double* __restrict__ V = pr.V;
  const int64_t k = pr.k, smax = pr.smax;
  const int64_t c0 = int64_t(it.blk) * CB;
  const int64_t rbeg = int64_t(it.ch) * pr.lrRch;
  const int64_t rend = min(k, rbeg + pr.lrRch);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  lr_d4 acc[2][NT];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[ct][nt] = lr_d4{0, 0, 0, 0};
  constexpr int QA = (RS * CB) / 256;
  constexpr int QU = (RS * NC + 255) / 256;
  double ra[QA], ru[QU];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int rr = e % RS, cc = e / RS;
      const int64_t rg = r0 + rr, cg = c0 + cc;
      ra[q] = (rg < rend && cg < smax) ? V[rg + cg * k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < QU; ++q) {
      const int e = threadIdx.x + 256 * q;
      int rr, i;
      if (LMAJ) { rr = e % RS; i = e / RS; } else { rr = e / NC; i = e % NC; }
      const int64_t rg = r0 + rr;
      double v = 0.0;
      if (e < RS * NC && rg < rend && i < N)
        v = LMAJ ? src[pr.offS * N + int64_t(i) * k + rg] : src[(pr.offS + rg) * N + i];
      ru[q] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = threadIdx.x + 256 * q;
      Vs[e / RS][e % RS] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QU; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < RS * NC) {
        if (LMAJ) Xs[e % RS][e / RS] = ru[q];
        else Xs[e / NC][e % NC] = ru[q];
      }
    }
  };
  if (rbeg < rend) {
    fetch(rbeg);
    stash();
  }
  __syncthreads();
  for (int64_t r0 = rbeg; r0 < rend; r0 += RS) {
    const bool more = r0 + RS < rend;
    if (more) fetch(r0 + RS);
#pragma unroll
    for (int ks = 0; ks < RS / 4; ++ks) {
      double a[2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) a[ct] = Vs[wv * 32 + ct * 16 + li][4 * ks + lk];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const double b = Xs[4 * ks + lk][nt * 16 + li];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          acc[ct][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ct], b, acc[ct][nt], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) stash();
    __syncthreads();
  }
  // result element (column 16 ct + 4 v + lane / 16 of the wave's 32, lambda 16 nt + lane % 16)
  double* dst = part + pr.lrPart + int64_t(it.ch) * pr.s * N;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = c0 + wv * 32 + ct * 16 + 4 * v + lk;
        const int lam = nt * 16 + li;
        if (j < smax && lam < N) dst[j * N + lam] = acc[ct][nt][v];
      }
}

// coef[j, i] = S_i[j] sum_ch part[ch][j][i] (row-major smax x N per problem);
// items: (problem, block of 256 entries).
__global__ void __launch_bounds__(256) k_lr_coef(const DevProb* __restrict__ P,
                                                 const Item* __restrict__ items, int N,
                                                 const double* __restrict__ part,
                                                 double* __restrict__ coef,
                                                 const Scal* __restrict__ sc) {
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t e = int64_t(it.blk) * 256 + threadIdx.x;
  if (e >= pr.smax * N) return;
  const int64_t j = e / N;
  const int i = int(e % N);
  double c = 0.0;
  for (int ch = 0; ch < pr.lrNch; ++ch) c += part[pr.lrPart + (int64_t(ch) * pr.s + j) * N + i];
  coef[pr.lrCoef + e] = c * pr.S[int64_t(sc[it.p * N + i].li) * pr.s + j];
}

static constexpr int LR_JC = 256;    // columns of V per expand block

template <int NC>
__global__ void __launch_bounds__(256) k_lr_expand(const DevProb* __restrict__ P,
                                                   const Item* __restrict__ items, int N,
                                                   const double* __restrict__ coef,
                                                   double* __restrict__ opart) {
  __shared__ double cs[LR_JC * NC];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t k = pr.k;
  const int64_t j0 = int64_t(it.ch) * LR_JC;
  const int jn = int(min<int64_t>(pr.smax - j0, LR_JC));
  for (int e = threadIdx.x; e < LR_JC * NC; e += 256) {
    const int jj = e / NC, i = e % NC;
    cs[e] = (jj < jn && i < N) ? coef[pr.lrCoef + (j0 + jj) * N + i] : 0.0;
  }
  __syncthreads();
  const int64_t r = int64_t(it.blk) * 256 + threadIdx.x;
  if (r >= k) return;
  double acc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) acc[i] = 0.0;
  const double* __restrict__ Vr = pr.V + r + j0 * k;
  int jj = 0;
  for (; jj + 4 <= jn; jj += 4) {
    const double v0 = Vr[int64_t(jj) * k], v1 = Vr[int64_t(jj + 1) * k];
    const double v2 = Vr[int64_t(jj + 2) * k], v3 = Vr[int64_t(jj + 3) * k];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      double a = acc[i];
      a = fma(v0, cs[jj * NC + i], a);
      a = fma(v1, cs[(jj + 1) * NC + i], a);
      a = fma(v2, cs[(jj + 2) * NC + i], a);
      a = fma(v3, cs[(jj + 3) * NC + i], a);
      acc[i] = a;
    }
  }
  for (; jj < jn; ++jj) {
    const double v0 = Vr[int64_t(jj) * k];
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] = fma(v0, cs[jj * NC + i], acc[i]);
  }
#pragma unroll
  for (int i = 0; i < NC; ++i)
    if (i < N) opart[pr.lrOpart + (int64_t(it.ch) * N + i) * k + r] = acc[i];
}

// STAGE 0 (the R^{-T} step of the v-update): q = R^{-1} t - beta_{i+1} v with
//   t stored lambda-major, and per-block partial squared norms of q;
//   TALL = false (Algorithm 4, the R^{-T} step of the u-update): the same
//   with alpha_i in place of beta_{i+1} and the partials in the beta array.
// STAGE 1 (the R^{-1} step): w = R^{-1} q / alpha, v = q / alpha and the x, e
//   recurrences (TALL); w = R^{-1} q / beta, u = q / beta (not TALL).
template <int NC, int STAGE, bool TALL>
__global__ void __launch_bounds__(256) k_lr_fin(const DevProb* __restrict__ P,
                                                const Item* __restrict__ items, int N,
                                                const double* __restrict__ src,
                                                const double* __restrict__ opart,
                                                double* __restrict__ q, double* __restrict__ v,
                                                double* __restrict__ w, double* __restrict__ x,
                                                double* __restrict__ e,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ pn, int init) {
  constexpr int FR = 256 / NC;
  __shared__ double sh[256];
  const Item it = items[blockIdx.x];
  const DevProb& pr = P[it.p];
  if (plan_stopped(pr)) return;
  const int64_t k = pr.k;
  const int i = threadIdx.x % NC;
  const int64_t r = int64_t(it.blk) * FR + threadIdx.x / NC;
  double nrm = 0.0;
  if (r < k && i < N) {
    double o = 0.0;
    for (int jc = 0; jc < pr.lrNjc; ++jc) o += opart[pr.lrOpart + (int64_t(jc) * N + i) * k + r];
    const Scal& S = sc[it.p * N + i];
    const double il = 1.0 / S.sqlam;
    const int64_t idx = (pr.offS + r) * N + i;
    if (STAGE == 0) {
      const double tv = src[pr.offS * N + int64_t(i) * k + r];
      const double nv = (tv - o) * il - (TALL ? S.beta_new : S.alpha) * v[idx];
      q[idx] = nv;
      nrm = nv * nv;
    } else {
      const double qv = src[idx];
      const double scale = TALL ? S.ialpha : S.ibeta;
      const double wr = (qv - o) * il * scale;
      v[idx] = qv * scale;
      w[idx] = wr;
      if (TALL) {
        if (init) {
          x[idx] = 0.0;
          e[idx] = wr;
        } else if (S.upd) {
          const double eo = e[idx];
          x[idx] += S.cx * eo;
          e[idx] = wr - S.ce * eo;
        }
      }
    }
  }
  if (STAGE != 0) return;
  sh[threadIdx.x] = nrm;
  __syncthreads();
  if (threadIdx.x < NC && int(threadIdx.x) < N) {
    double s = 0.0;
    for (int rr = 0; rr < FR; ++rr) s += sh[rr * NC + threadIdx.x];
    pn[((TALL ? pr.pnQ : pr.pnN) + it.blk) * N + threadIdx.x] = s;
  }
}

template <int NC>
static int lr_apply_nc(int stage, int tall, const DevProb* P, const Item* itP, int nP,
                       const Item* itC, int nC, const Item* itE, int nE, const Item* itF, int nF,
                       int N, const double* src, double* part, double* coef, double* opart,
                       double* q, double* v, double* w, double* x, double* e, const Scal* sc,
                       double* pn, int init, hipStream_t st) {
  constexpr int CPW = NC >= 32 ? 2 : 4;
  if (nP > 0) {
    // t (stage 0) is stored lambda-major, q (stage 1) row-major
    if (NC >= 16) {
      const dim3 g = dim3(unsigned(((nP + 7) / 8) * 8));
      if (stage == 0)
        hipLaunchKernelGGL((k_lr_proj_mfma<NC >= 16 ? NC : 16, true>), g, dim3(256), 0, st, P, itP, nP,
                           N, src, part);
      else
        hipLaunchKernelGGL((k_lr_proj_mfma<NC >= 16 ? NC : 16, false>), g, dim3(256), 0, st, P, itP,
                           nP, N, src, part);
    } else if (stage == 0) {
      hipLaunchKernelGGL((k_lr_proj<NC, CPW, true>), dim3(unsigned(nP)), dim3(256), 0, st, P, itP, N,
                         src, part);
    } else {
      hipLaunchKernelGGL((k_lr_proj<NC, CPW, false>), dim3(unsigned(nP)), dim3(256), 0, st, P, itP, N,
                         src, part);
    }
    TIK_LAUNCHED("k_lr_proj");
    hipLaunchKernelGGL(k_lr_coef, dim3(unsigned(nC)), dim3(256), 0, st, P, itC, N, part, coef, sc);
    TIK_LAUNCHED("k_lr_coef");
  }
  if (nE > 0) {
    hipLaunchKernelGGL(k_lr_expand<NC>, dim3(unsigned(nE)), dim3(256), 0, st, P, itE, N, coef, opart);
    TIK_LAUNCHED("k_lr_expand");
  }
  if (nF > 0) {
    if (stage == 0) {
      if (tall)
        hipLaunchKernelGGL((k_lr_fin<NC, 0, true>), dim3(unsigned(nF)), dim3(256), 0, st, P, itF, N, src,
                           opart, q, v, w, x, e, sc, pn, init);
      else
        hipLaunchKernelGGL((k_lr_fin<NC, 0, false>), dim3(unsigned(nF)), dim3(256), 0, st, P, itF, N,
                           src, opart, q, v, w, x, e, sc, pn, init);
    } else {
      if (tall)
        hipLaunchKernelGGL((k_lr_fin<NC, 1, true>), dim3(unsigned(nF)), dim3(256), 0, st, P, itF, N, src,
                           opart, q, v, w, x, e, sc, pn, init);
      else
        hipLaunchKernelGGL((k_lr_fin<NC, 1, false>), dim3(unsigned(nF)), dim3(256), 0, st, P, itF, N,
                           src, opart, q, v, w, x, e, sc, pn, init);
    }
    TIK_LAUNCHED("k_lr_fin");
  }
  return TIK_OK;
}

int launch_lr_apply(int nc, int stage, int tall, const DevProb* P, const LrItems& it, int N,
                    const double* src, const LrBufs& lb, double* q, double* v, double* w, double* x,
                    double* e, const Scal* sc, double* pn, int init, hipStream_t st) {
  switch (nc) {
#define TIK_LR_CASE(NCV)                                                                         \
  case NCV:                                                                                      \
    return lr_apply_nc<NCV>(stage, tall, P, it.P, it.nP, it.C, it.nC, it.E, it.nE, it.F, it.nF, N, \
                          src, lb.part, lb.coef, lb.opart, q, v, w, x, e, sc, pn, init, st);
    TIK_LR_CASE(1)
    TIK_LR_CASE(2)
    TIK_LR_CASE(4)
    TIK_LR_CASE(8)
    TIK_LR_CASE(16)
    TIK_LR_CASE(32)
#undef TIK_LR_CASE
  }
  set_error("internal: lambda batch wider than 32");
  return TIK_ENOTSUP;
}

}  // namespace tik
