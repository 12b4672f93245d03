/* Gradient of the Tikhonov objective in extended precision.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle): nothing in the product
 * links or loads this file's library.
 *
 * For candidate solutions X (n x N, column-major, ld n) of
 * min ||A x - b||^2 + lam ||x||^2 (eq. regLLS) this computes
 *     G[:, i] = A^T (b - A X[:, i]) - lam_i X[:, i],
 * the negated half-gradient, whose norm bounds the forward error through the
 * normal equations (A^T A + lam I) x_lam = A^T b.  Both products accumulate in
 * long double (64-bit significand on x86), so the rounding error of G stays
 * about 2^-11 below that of an FP64 evaluation.
 *
 * A is m x n column-major with leading dimension lda, stored as float
 * (f32 != 0) or double.  Parallel over row blocks (first product) and column
 * blocks (second product) with OpenMP; no reordering beyond that.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RB 256
#define CB 16

static inline long double a_at(const void* A, int f32, int64_t lda, int64_t r, int64_t c) {
  return f32 ? (long double)((const float*)A)[r + c * lda] : (long double)((const double*)A)[r + c * lda];
}

int oracle_tik_gradient(const void* A, int f32, int64_t m, int64_t n, int64_t lda,
                        const double* b, const double* X, const double* lams, int N,
                        double* G) {
  if (N < 1 || m < 1 || n < 1) return -1;
  long double* R = (long double*)malloc(sizeof(long double) * (size_t)m * (size_t)N);   /* m x N row-major */
  long double* Xt = (long double*)malloc(sizeof(long double) * (size_t)n * (size_t)N);  /* n x N row-major */
  if (!R || !Xt) {
    free(R);
    free(Xt);
    return -2;
  }
  for (int64_t j = 0; j < n; ++j)
    for (int i = 0; i < N; ++i) Xt[j * N + i] = (long double)X[j + (int64_t)i * n];

  /* R = b - A X, one block of rows per task */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r0 = 0; r0 < m; r0 += RB) {
    const int64_t r1 = r0 + RB < m ? r0 + RB : m;
    long double* Rb = R + r0 * N;
    for (int64_t r = r0; r < r1; ++r)
      for (int i = 0; i < N; ++i) Rb[(r - r0) * N + i] = (long double)b[r];
    for (int64_t j = 0; j < n; ++j) {
      const long double* xj = Xt + j * N;
      for (int64_t r = r0; r < r1; ++r) {
        const long double a = a_at(A, f32, lda, r, j);
        long double* rr = Rb + (r - r0) * N;
        for (int i = 0; i < N; ++i) rr[i] -= a * xj[i];
      }
    }
  }

  /* G = A^T R - lam X, one block of columns per task */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c0 = 0; c0 < n; c0 += CB) {
    const int64_t c1 = c0 + CB < n ? c0 + CB : n;
    long double acc[CB][64];
    const int NB = N < 64 ? N : 64;
    for (int i0 = 0; i0 < N; i0 += NB) {
      const int ni = (N - i0) < NB ? (N - i0) : NB;
      for (int64_t c = c0; c < c1; ++c)
        for (int i = 0; i < ni; ++i) acc[c - c0][i] = 0.0L;
      for (int64_t r = 0; r < m; ++r) {
        const long double* rr = R + r * N + i0;
        for (int64_t c = c0; c < c1; ++c) {
          const long double a = a_at(A, f32, lda, r, c);
          for (int i = 0; i < ni; ++i) acc[c - c0][i] += a * rr[i];
        }
      }
      for (int64_t c = c0; c < c1; ++c)
        for (int i = 0; i < ni; ++i) {
          const long double x = Xt[c * N + i0 + i];
          G[c + (int64_t)(i0 + i) * n] = (double)(acc[c - c0][i] - (long double)lams[i0 + i] * x);
        }
    }
  }
  free(R);
  free(Xt);
  return 0;
}
