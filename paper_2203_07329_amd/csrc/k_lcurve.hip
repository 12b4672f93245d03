// L-curve of Section 4.3 (Fig. 4): for every problem and lambda, the solution
// norm ||x_lam||_2 and the residual norm ||A x_lam - b||_2 in FP64, from the
// solutions tik_lsqr_batch wrote; the corner of the log-log curve is chosen on
// the host (tik_lcurve_corner in tik_api.hip).
//
// One pass over each A serves all lambdas of a group of up to 32: a block owns
// 256 consecutive rows and a chunk of columns; each thread keeps one row's
// products with every x of the group, the x rows of the chunk being staged
// through LDS 64 columns at a time.  Column chunks write partial products; a
// second kernel sums them in a fixed order and reduces the norms per lambda.
#include "tik_internal.h"

namespace tik {

static constexpr int LC_ROWS = 256;   // rows of A per block (one per thread)
static constexpr int LC_KC = 64;      // columns of A staged per LDS step

struct LcProb {
  const void* A;
  const double* b;
  const double* X;   // n x N column-major (ld n) for this problem
  int64_t m, n, lda;
  int32_t a_f32, nch;
  int64_t cchunk;    // columns per chunk
  int64_t part;      // offset of this problem's partials (nch x m x NG)
  int64_t pn;        // first norm block of this problem (row blocks, then column blocks)
  int32_t nrb, ncb;  // row blocks of 256 and column blocks of 256
};

struct LcItem {
  int32_t p, rb, ch, pad;
};

// part[ch][r][i] = sum over the chunk's columns c of A[r, c] x_{l0 + i}[c]
template <typename TA, int NG>
__global__ void __launch_bounds__(LC_ROWS) k_lc_prod(const LcProb* __restrict__ P,
                                                     const LcItem* __restrict__ items, int l0,
                                                     int ng, double* __restrict__ part) {
  __shared__ double xs[LC_KC][NG + 1];
  const LcItem it = items[blockIdx.x];
  const LcProb& pr = P[it.p];
  const TA* __restrict__ A = static_cast<const TA*>(pr.A);
  const int64_t r = int64_t(it.rb) * LC_ROWS + threadIdx.x;
  const int64_t c0 = int64_t(it.ch) * pr.cchunk;
  const int64_t c1 = min(pr.n, c0 + pr.cchunk);
  double acc[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) acc[i] = 0.0;
  for (int64_t k0 = c0; k0 < c1; k0 += LC_KC) {
    const int kc = int(min<int64_t>(LC_KC, c1 - k0));
    for (int e = threadIdx.x; e < LC_KC * NG; e += LC_ROWS) {
      const int kk = e % LC_KC, i = e / LC_KC;
      xs[kk][i] = (kk < kc && i < ng) ? pr.X[(k0 + kk) + int64_t(l0 + i) * pr.n] : 0.0;
    }
    __syncthreads();
    if (r < pr.m) {
      const TA* __restrict__ col = A + r + k0 * pr.lda;
      for (int kk = 0; kk < kc; ++kk) {
        const double a = double(col[int64_t(kk) * pr.lda]);
#pragma unroll
        for (int i = 0; i < NG; ++i) acc[i] = fma(a, xs[kk][i], acc[i]);
      }
    }
    __syncthreads();
  }
  if (r < pr.m) {
    double* dst = part + pr.part + (int64_t(it.ch) * pr.m + r) * NG;
#pragma unroll
    for (int i = 0; i < NG; ++i) dst[i] = acc[i];
  }
}

// Per block: partial sums of (b - A x)^2 over 256 rows (row blocks) or of x^2
// over 256 entries of x (column blocks), for each lambda of the group.
template <int NG>
__global__ void __launch_bounds__(256) k_lc_sq(const LcProb* __restrict__ P,
                                               const LcItem* __restrict__ items, int l0, int ng,
                                               const double* __restrict__ part,
                                               double* __restrict__ pn) {
  __shared__ double sh[4][NG];
  const LcItem it = items[blockIdx.x];
  const LcProb& pr = P[it.p];
  const bool rowblk = it.ch == 0;
  const int64_t r = int64_t(it.rb) * 256 + threadIdx.x;
  double v[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) v[i] = 0.0;
  if (rowblk && r < pr.m) {
    const double br = pr.b[r];
    // the row's NG partial products of each chunk are contiguous: read them
    // chunk by chunk (each sum still runs over the chunks in order)
    double ax[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) ax[i] = 0.0;
    for (int ch = 0; ch < pr.nch; ++ch) {
      const double* src = part + pr.part + (int64_t(ch) * pr.m + r) * NG;
#pragma unroll
      for (int i = 0; i < NG; ++i) ax[i] += src[i];
    }
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const double d = br - ax[i];
      v[i] = d * d;
    }
  } else if (!rowblk && r < pr.n) {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const double x = i < ng ? pr.X[r + int64_t(l0 + i) * pr.n] : 0.0;
      v[i] = x * x;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) sh[wv][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NG) {
    const int i = threadIdx.x;
    const int64_t blk = pr.pn + (rowblk ? it.rb : pr.nrb + it.rb);
    pn[blk * NG + i] = sh[0][i] + sh[1][i] + sh[2][i] + sh[3][i];
  }
}

// One block per (problem, lambda of the group): the two square roots.
template <int NG>
__global__ void __launch_bounds__(256) k_lc_fin(const LcProb* __restrict__ P, int N, int l0, int ng,
                                                const double* __restrict__ pn,
                                                double* __restrict__ xnorm,
                                                double* __restrict__ rnorm) {
  __shared__ double sh[2][4];
  const int p = blockIdx.x / ng, i = blockIdx.x % ng;
  const LcProb& pr = P[p];
  double sr = 0.0, sx = 0.0;
  for (int b = threadIdx.x; b < pr.nrb; b += 256) sr += pn[(pr.pn + b) * NG + i];
  for (int b = threadIdx.x; b < pr.ncb; b += 256) sx += pn[(pr.pn + pr.nrb + b) * NG + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    sx += __shfl_xor(sx, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wv] = sr;
    sh[1][wv] = sx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const size_t g = size_t(p) * N + l0 + i;
    if (rnorm) rnorm[g] = sqrt(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3]);
    if (xnorm) xnorm[g] = sqrt(sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
  }
}

namespace {

struct LcPlan {
  std::vector<LcProb> P;
  std::vector<LcItem> prod, sq;
  int64_t tot_part = 0, tot_pn = 0;
};

constexpr int LC_NG = 32;   // lambdas per pass over A

void lc_plan(const tik_problem* p, int32_t nprob, double* const* X, LcPlan& pl) {
  pl = LcPlan();
  int64_t work = 0;
  for (int k = 0; k < nprob; ++k) work += cdiv(p[k].m, LC_ROWS) * p[k].n;
  // columns per chunk: about 2048 product blocks over the whole batch, each
  // at least 512 columns (a multiple of the LDS step)
  const int64_t target = std::max<int64_t>(512, cdiv(cdiv(work, 2048), LC_KC) * LC_KC);
  for (int k = 0; k < nprob; ++k) {
    LcProb d = {};
    d.A = p[k].A;
    d.b = p[k].b;
    d.X = X ? X[k] : nullptr;
    d.m = p[k].m;
    d.n = p[k].n;
    d.lda = p[k].lda;
    d.a_f32 = p[k].a_dtype == TIK_F32;
    d.nch = int32_t(cdiv(d.n, target));
    d.cchunk = cdiv(cdiv(d.n, d.nch), LC_KC) * LC_KC;
    d.nch = int32_t(cdiv(d.n, d.cchunk));
    d.part = pl.tot_part;
    d.nrb = int32_t(cdiv(d.m, 256));
    d.ncb = int32_t(cdiv(d.n, 256));
    d.pn = pl.tot_pn;
    pl.tot_part += int64_t(d.nch) * d.m * LC_NG;
    pl.tot_pn += d.nrb + d.ncb;
    for (int ch = 0; ch < d.nch; ++ch)
      for (int rb = 0; rb < int(cdiv(d.m, LC_ROWS)); ++rb) pl.prod.push_back({k, rb, ch, 0});
    for (int rb = 0; rb < d.nrb; ++rb) pl.sq.push_back({k, rb, 0, 0});
    for (int cb = 0; cb < d.ncb; ++cb) pl.sq.push_back({k, cb, 1, 0});
    pl.P.push_back(d);
  }
}

size_t lc_take(Arena& a, const LcPlan& pl, LcProb** P, LcItem** prod, LcItem** sq, double** part,
               double** pn) {
  *P = a.take<LcProb>(pl.P.size());
  *prod = a.take<LcItem>(pl.prod.size());
  *sq = a.take<LcItem>(pl.sq.size());
  *part = a.take<double>(size_t(pl.tot_part));
  *pn = a.take<double>(size_t(pl.tot_pn) * LC_NG);
  return a.used;
}

}  // namespace

int lcurve_bytes(const tik_problem* p, int32_t nprob, size_t* bytes) {
  LcPlan pl;
  lc_plan(p, nprob, nullptr, pl);
  Arena a;
  LcProb* P;
  LcItem *prod, *sq;
  double *part, *pn;
  *bytes = lc_take(a, pl, &P, &prod, &sq, &part, &pn) + 256;
  return TIK_OK;
}

int lcurve_run(const tik_problem* p, int32_t nprob, int32_t N, double* const* X, double* xnorm,
               double* rnorm, void* dws, size_t dws_bytes, hipStream_t st) {
  const bool f32 = p[0].a_dtype == TIK_F32;
  for (int k = 1; k < nprob; ++k)
    if ((p[k].a_dtype == TIK_F32) != f32) {
      set_error("tik_lcurve: all problems of one call must share A's storage type");
      return TIK_EINVAL;
    }
  LcPlan pl;
  lc_plan(p, nprob, X, pl);
  Arena a;
  a.base = static_cast<char*>(dws);
  a.cap = dws_bytes;
  LcProb* P;
  LcItem *prod, *sq;
  double *part, *pn;
  lc_take(a, pl, &P, &prod, &sq, &part, &pn);
  if (!a.fits()) {
    set_error("tik_lcurve: workspace too small");
    return TIK_EWORKSPACE;
  }
  TIK_HIP(hipMemcpyAsync(P, pl.P.data(), pl.P.size() * sizeof(LcProb), hipMemcpyHostToDevice, st));
  TIK_HIP(hipMemcpyAsync(prod, pl.prod.data(), pl.prod.size() * sizeof(LcItem), hipMemcpyHostToDevice, st));
  TIK_HIP(hipMemcpyAsync(sq, pl.sq.data(), pl.sq.size() * sizeof(LcItem), hipMemcpyHostToDevice, st));
  for (int l0 = 0; l0 < N; l0 += LC_NG) {
    const int ng = std::min(LC_NG, N - l0);
    if (f32)
      hipLaunchKernelGGL((k_lc_prod<float, LC_NG>), dim3(unsigned(pl.prod.size())), dim3(LC_ROWS), 0, st,
                         P, prod, l0, ng, part);
    else
      hipLaunchKernelGGL((k_lc_prod<double, LC_NG>), dim3(unsigned(pl.prod.size())), dim3(LC_ROWS), 0,
                         st, P, prod, l0, ng, part);
    TIK_LAUNCHED("k_lc_prod");
    hipLaunchKernelGGL((k_lc_sq<LC_NG>), dim3(unsigned(pl.sq.size())), dim3(256), 0, st, P, sq, l0, ng,
                       part, pn);
    TIK_LAUNCHED("k_lc_sq");
    hipLaunchKernelGGL((k_lc_fin<LC_NG>), dim3(unsigned(nprob * ng)), dim3(256), 0, st, P, N, l0, ng, pn,
                       xnorm, rnorm);
    TIK_LAUNCHED("k_lc_fin");
  }
  // the plan tables were copied from host vectors that die on return
  TIK_HIP(hipStreamSynchronize(st));
  return TIK_OK;
}

}  // namespace tik
