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

// ---------------------------------------------------------------- Gram ------
// C (n x n, ld n) = Z^T Z with Z K x n column-major (ld ldz).  Upper tile pairs
// are computed and written to both triangles.
__global__ void __launch_bounds__(256) k_syrk(const double* __restrict__ Z, int64_t K, int64_t n,
                                              int64_t ldz, double* __restrict__ C, int nt) {
  // map blockIdx.x to tile pair (ti <= tj)
  int t = blockIdx.x, ti = 0;
  while (t >= nt - ti) { t -= nt - ti; ++ti; }
  const int tj = ti + t;
  __shared__ double Za[16][64 + 1];
  __shared__ double Zb[16][64 + 1];
  const int tid = threadIdx.x;
  const int ta = tid & 15, tb = tid >> 4;
  const int64_t a0 = int64_t(ti) * 64, b0 = int64_t(tj) * 64;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e & 15, cc = e >> 4;
      const int64_t kg = k0 + kk;
      Za[kk][cc] = (kg < K && a0 + cc < n) ? Z[kg + (a0 + cc) * ldz] : 0.0;
      Zb[kk][cc] = (kg < K && b0 + cc < n) ? Z[kg + (b0 + cc) * ldz] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double x[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = Za[kk][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = Zb[kk][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t a = a0 + ta + 16 * i, b = b0 + tb + 16 * j;
      if (a < n && b < n) {
        C[a + b * n] = acc[i][j];
        C[b + a * n] = acc[i][j];
      }
    }
}

// ----------------------------------------------------- shifted copies -------
__global__ void k_shift_copy(const double* __restrict__ C, int64_t n, const double* __restrict__ lams,
                             double* __restrict__ R) {
  const int64_t mat = blockIdx.y;
  const int64_t nn = n * n;
  double* Rm = R + mat * nn;
  const double lam = lams[mat];
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nn;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e % n, c = e / n;
    Rm[e] = C[e] + (r == c ? lam : 0.0);
  }
}

// --------------------------------------------- diagonal block: factor+invert --
__global__ void __launch_bounds__(256) k_potrf_diag(double* __restrict__ R, int64_t n, int64_t k0,
                                                    double* __restrict__ Dinv, int32_t* notpd) {
  const int64_t mat = blockIdx.x;
  double* Rm = R + mat * n * n;
  const int kb = int(min<int64_t>(NB, n - k0));
  __shared__ double Am[NB][NB + 1];
  __shared__ double Ai[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    Am[i][j] = (i < kb && j < kb && i <= j) ? Rm[(k0 + i) + (k0 + j) * n] : 0.0;
    Ai[i][j] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    if (tid == 0) {
      double d = Am[k][k];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        d = 1.0;
      }
      Am[k][k] = sqrt(d);
    }
    __syncthreads();
    const double piv = Am[k][k];
    for (int j = k + 1 + tid; j < kb; j += 256) Am[k][j] /= piv;
    __syncthreads();
    const int rem = kb - k - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = k + 1 + e % rem, j = k + 1 + e / rem;
      if (i <= j) Am[i][j] -= Am[k][i] * Am[k][j];
    }
    __syncthreads();
  }
  // inverse of the upper-triangular block, column by column
  for (int j = 0; j < kb; ++j) {
    const double djj = Am[j][j];
    if (tid < j) {
      const int i = tid;
      double s = 0.0;
      for (int t = i; t < j; ++t) s += Ai[i][t] * Am[t][j];
      Ai[i][j] = -s / djj;
    } else if (tid == j) {
      Ai[j][j] = 1.0 / djj;
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e % kb, j = e / kb;
    Rm[(k0 + i) + (k0 + j) * n] = (i <= j) ? Am[i][j] : 0.0;
  }
  double* D = Dinv + (mat * cdiv(n, NB) + k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e % NB, j = e / NB;
    D[e] = (i < kb && j < kb) ? Ai[i][j] : 0.0;
  }
  if (tid == 0 && bad) notpd[mat] = 1;
}

// R[k0:k0+kb, cols] = D^T R[k0:k0+kb, cols] for the 64-column tile blockIdx.x
// right of the diagonal block (D = inverse of the diagonal block).
__global__ void __launch_bounds__(256) k_trsm_panel(double* __restrict__ R, int64_t n, int64_t k0,
                                                    const double* __restrict__ Dinv) {
  const int64_t mat = blockIdx.y;
  double* Rm = R + mat * n * n;
  const int kb = int(min<int64_t>(NB, n - k0));
  const int64_t c0 = k0 + kb + int64_t(blockIdx.x) * 64;
  __shared__ double D[NB][NB + 1];
  __shared__ double P[NB][64 + 1];
  const int tid = threadIdx.x;
  const double* Dm = Dinv + (mat * cdiv(n, NB) + k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += 256) D[e % NB][e / NB] = Dm[e];
  for (int e = tid; e < NB * 64; e += 256) {
    const int i = e % NB, c = e / NB;
    P[i][c] = (i < kb && c0 + c < n) ? Rm[(k0 + i) + (c0 + c) * n] : 0.0;
  }
  __syncthreads();
  const int ti = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int t = 0; t < kb; ++t) {
    double d[4], p[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) d[a] = D[t][ti + 16 * a];   // (D^T)[i][t] = D[t][i]
#pragma unroll
    for (int b = 0; b < 4; ++b) p[b] = P[t][tc + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(d[a], p[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ti + 16 * a;
      const int64_t c = c0 + tc + 16 * b;
      if (i < kb && c < n) Rm[(k0 + i) + c * n] = acc[a][b];
    }
}

// Trailing update of the upper tiles: R[a, b] -= R[k, a]^T R[k, b] over the
// panel rows k (tile pair blockIdx.x, a <= b, tiles counted from k0 + kb).
__global__ void __launch_bounds__(256) k_syrk_trail(double* __restrict__ R, int64_t n, int64_t k0,
                                                    int nt) {
  const int64_t mat = blockIdx.y;
  double* Rm = R + mat * n * n;
  const int kb = int(min<int64_t>(NB, n - k0));
  int t = blockIdx.x, ta = 0;
  while (t >= nt - ta) { t -= nt - ta; ++ta; }
  const int tb = ta + t;
  const int64_t base = k0 + kb;
  const int64_t a0 = base + int64_t(ta) * 64, b0 = base + int64_t(tb) * 64;
  __shared__ double Pa[NB][64 + 1];
  __shared__ double Pb[NB][64 + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * 64; e += 256) {
    const int i = e % NB, c = e / NB;
    Pa[i][c] = (i < kb && a0 + c < n) ? Rm[(k0 + i) + (a0 + c) * n] : 0.0;
    Pb[i][c] = (i < kb && b0 + c < n) ? Rm[(k0 + i) + (b0 + c) * n] : 0.0;
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  for (int k = 0; k < kb; ++k) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = Pa[k][tx + 16 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = Pb[k][ty + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t a = a0 + tx + 16 * i, b = b0 + ty + 16 * j;
      if (a < n && b < n) Rm[a + b * n] -= acc[i][j];
    }
}

// Tmp[rows of tile blockIdx.x, 0:lb] = Rinv[rows, 0:l0] R[0:l0, l0:l0+lb]
// (Rinv upper triangular, already stored in columns < l0).
__global__ void __launch_bounds__(256) k_trinv_mul(const double* __restrict__ R, int64_t n,
                                                   int64_t l0, double* __restrict__ Tmp) {
  const int64_t mat = blockIdx.y;
  const double* Rm = R + mat * n * n;
  const int lb = int(min<int64_t>(NB, n - l0));
  const int64_t r0 = int64_t(blockIdx.x) * 64;
  __shared__ double Ri[64][16 + 1];
  __shared__ double Rb[16][NB + 1];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int64_t k0 = r0; k0 < l0; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int i = e & 63, kk = e >> 6;
      const int64_t r = r0 + i, k = k0 + kk;
      Ri[i][kk] = (r < l0 && k < l0) ? Rm[r + k * n] : 0.0;
    }
    for (int e = tid; e < 16 * NB; e += 256) {
      const int kk = e & 15, c = e >> 4;
      const int64_t k = k0 + kk;
      Rb[kk][c] = (k < l0 && c < lb) ? Rm[k + (l0 + c) * n] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double x[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = Ri[tr + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = Rb[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* Tm = Tmp + mat * n * NB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = r0 + tr + 16 * i;
      const int c = tc + 16 * j;
      if (r < l0 && c < lb) Tm[r + int64_t(c) * n] = acc[i][j];
    }
}

// Block column l of Rinv: rows above the diagonal block get -Tmp D_l, the
// diagonal block gets D_l, rows below get zero (the lower triangle).
__global__ void __launch_bounds__(256) k_trinv_fin(double* __restrict__ R, int64_t n, int64_t l0,
                                                   const double* __restrict__ Tmp,
                                                   const double* __restrict__ Dinv) {
  const int64_t mat = blockIdx.y;
  double* Rm = R + mat * n * n;
  const int lb = int(min<int64_t>(NB, n - l0));
  const int64_t r0 = int64_t(blockIdx.x) * 64;
  const int tid = threadIdx.x;
  const double* Dm = Dinv + (mat * cdiv(n, NB) + l0 / NB) * NB * NB;
  if (r0 >= l0 + lb || r0 == l0) {
    // below the diagonal block (zeros) or the diagonal block itself
    for (int e = tid; e < 64 * NB; e += 256) {
      const int i = e & 63, c = e >> 6;
      const int64_t r = r0 + i;
      if (r < n && c < lb) {
        double v = 0.0;
        if (r0 == l0 && i <= c) v = Dm[i + c * NB];
        Rm[r + (l0 + c) * n] = v;
      }
    }
    return;
  }
  __shared__ double Tt[64][NB + 1];
  __shared__ double D[NB][NB + 1];
  const double* Tm = Tmp + mat * n * NB;
  for (int e = tid; e < 64 * NB; e += 256) {
    const int i = e & 63, c = e >> 6;
    const int64_t r = r0 + i;
    Tt[i][c] = (r < l0 && c < lb) ? Tm[r + int64_t(c) * n] : 0.0;
  }
  for (int e = tid; e < NB * NB; e += 256) D[e % NB][e / NB] = Dm[e];
  __syncthreads();
  const int tr = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int t = 0; t < lb; ++t) {
    double x[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = Tt[tr + 16 * i][t];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = D[t][tc + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = r0 + tr + 16 * i;
      const int c = tc + 16 * j;
      if (r < l0 && c < lb) Rm[r + (l0 + c) * n] = -acc[i][j];
    }
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
int launch_syrk(const double* Z, int64_t K, int64_t n, int64_t ldz, double* C, hipStream_t st) {
  const int nt = int(cdiv(n, 64));
  ProfScope ps("gram", st);
  hipLaunchKernelGGL(k_syrk, dim3(unsigned(nt * (nt + 1) / 2)), dim3(256), 0, st, Z, K, n, ldz,
                     C, nt);
  TIK_LAUNCHED("k_syrk");
  return TIK_OK;
}

// R (nb_mat matrices n x n) <- inverse of chol(C + lams[j] I); notpd[j] = 1 on
// breakdown.  Dinv: nb_mat * ceil(n/64) * 64 * 64 doubles; Tmp: nb_mat * n * 64.
int launch_chol_inv_batched(const double* C, int64_t n, const double* lams, int32_t nb_mat,
                            double* R, double* Dinv, double* Tmp, int32_t* notpd,
                            hipStream_t st) {
  const int64_t nblk = cdiv(n, NB);
  {
    ProfScope ps("chol", st);
    const unsigned gx = unsigned(std::min<int64_t>(cdiv(n * n, 256), 4096));
    hipLaunchKernelGGL(k_shift_copy, dim3(gx, unsigned(nb_mat)), dim3(256), 0, st, C, n, lams, R);
    TIK_LAUNCHED("k_shift_copy");
    for (int64_t kb = 0; kb < nblk; ++kb) {
      const int64_t k0 = kb * NB;
      hipLaunchKernelGGL(k_potrf_diag, dim3(unsigned(nb_mat)), dim3(256), 0, st, R, n, k0, Dinv,
                         notpd);
      TIK_LAUNCHED("k_potrf_diag");
      const int64_t rest = n - k0 - std::min<int64_t>(NB, n - k0);
      if (rest > 0) {
        const int nt = int(cdiv(rest, 64));
        hipLaunchKernelGGL(k_trsm_panel, dim3(unsigned(nt), unsigned(nb_mat)), dim3(256), 0, st,
                           R, n, k0, Dinv);
        TIK_LAUNCHED("k_trsm_panel");
        hipLaunchKernelGGL(k_syrk_trail, dim3(unsigned(nt * (nt + 1) / 2), unsigned(nb_mat)),
                           dim3(256), 0, st, R, n, k0, nt);
        TIK_LAUNCHED("k_syrk_trail");
      }
    }
  }
  {
    ProfScope ps("trinv", st);
    for (int64_t lb = 0; lb < nblk; ++lb) {
      const int64_t l0 = lb * NB;
      if (l0 > 0) {
        hipLaunchKernelGGL(k_trinv_mul, dim3(unsigned(cdiv(l0, 64)), unsigned(nb_mat)), dim3(256),
                           0, st, R, n, l0, Tmp);
        TIK_LAUNCHED("k_trinv_mul");
      }
      hipLaunchKernelGGL(k_trinv_fin, dim3(unsigned(cdiv(n, 64)), unsigned(nb_mat)), dim3(256), 0,
                         st, R, n, l0, Tmp, Dinv);
      TIK_LAUNCHED("k_trinv_fin");
    }
  }
  return TIK_OK;
}

}  // namespace tik
