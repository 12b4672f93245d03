// Matrix-core (MFMA) versions of the two batched products of an LSQR step,
// used when 16 or 32 lambdas share each pass over A:
//   gemm_n:  u~_top = A W - ucoef u~_top       (m x N, contraction over the n columns)
//   gemm_t:  partial A^T U over a row chunk     (n x N, contraction over the m rows)
// FP64 uses v_mfma_f64_16x16x4_f64, FP32 uses v_mfma_f32_16x16x4_f32.  Both
// take one operand element per lane: A-operand element (i = lane % 16,
// k = lane / 16), B-operand element (k = lane / 16, j = lane % 16).  The
// 16 x 16 result sits in four registers per lane: column j = lane % 16, row
// i = 4 v + lane / 16 for FP64 and i = 4 (lane / 16) + v for FP32 (v = 0..3).
#include "tik_internal.h"

#include <map>
#include <mutex>
#include <tuple>

namespace tik {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename TC>
struct Mfma;

template <>
struct Mfma<double> {
  using acc_t = mf_d4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mfma<float> {
  using acc_t = mf_f4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// ------------------------------------------------------------------ gemm_n --
// Block = 4 waves x 16 RT rows = 64 RT rows of one problem, all NC lambdas.
// A is read straight into A-operand registers (16 consecutive rows of 4
// columns per load: whole 64/128-byte lines); W is staged through LDS KC
// columns at a time.  RT = 2 (128-row blocks) keeps the registers low for tall
// problems; RT = 4 (256 rows) halves the re-reads of W where the A rows are
// few and W is long (wide problems).  The plan's rows per block must match.
// EPI 0: LSQR update of u~_top with partial squared norms; EPI 1: store A W;
// EPI 2: store the partial product over column chunk it.ch (wide problems).
template <typename TA, typename TC, int NC, int EPI, int RT>
__global__ void __launch_bounds__(256, RT == 2 ? 3 : 2) k_gemm_n_mfma(const DevProb* __restrict__ P,
                                                     const Item* __restrict__ items, int N,
                                                     const TC* __restrict__ W,
                                                     TC* __restrict__ ut, double* __restrict__ out,
                                                     const Scal* __restrict__ sc,
                                                     double* __restrict__ pnN,
                                                     const DevProb* __restrict__ P2,
                                                     TC* __restrict__ part2) {
  using M = Mfma<TC>;
  constexpr int NT = NC / 16;
  // columns per chunk: 128 bytes of each row (64 where FP64 operands of
  // 256-row blocks would not fit the registers)
  constexpr int KC = (sizeof(TA) == 8 || (sizeof(TC) == 8 && RT == 4)) ? 16 : 32;
  constexpr int WP = NC + 2;
  constexpr int QW = (KC * NC + 255) / 256;     // W elements per thread and chunk
  __shared__ TC Ws[2][KC][WP];
  __shared__ double nred[4][NC];
  const Item it = items[blockIdx.x];
  // EPI 3: the row blocks (EPI 0) and, flagged by it.j, the column pieces of
  // the last round's row blocks (EPI 2 on descriptor P2, stored to part2) in
  // one launch, listed after the row blocks so that they fill the compute
  // units the row blocks' last round leaves idle
  const bool piece = EPI == 3 && it.j != 0;
  const bool ep0 = EPI == 0 || (EPI == 3 && !piece);
  const DevProb& pr = piece ? *P2 : P[it.p];
  if (pr.live && *pr.live == 0) return;   // every solve of the plan has stopped
  const TA* __restrict__ A = static_cast<const TA*>(pr.A);
  const int64_t m = pr.m, n = pr.n, lda = pr.lda;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = int64_t(it.blk) * (64 * RT) + wv * (16 * RT);
  const int64_t kbeg = int64_t(it.ch) * pr.cchunk;
  const int64_t kend = min(n, kbeg + pr.cchunk);
  typename M::acc_t acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = typename M::acc_t{0, 0, 0, 0};
  // The A operands and the W rows of the next chunk are loaded into registers
  // while the matrix cores work on the current chunk; W is double-buffered in
  // LDS, so one barrier per chunk suffices.
  auto load_a = [&](int64_t k0, TA (&dst)[RT][KC / 4]) {   // kept as stored, widened at use
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int64_t col = k0 + 4 * ks + lk;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int64_t row = row0 + rt * 16 + li;
        dst[rt][ks] = (row < m && col < kend) ? A[row + col * lda] : TA(0);
      }
    }
  };
  auto load_w = [&](int64_t k0, TC (&dst)[QW]) {
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int kk = e / NC, i = e % NC;
      const int64_t kg = k0 + kk;
      dst[q] = (e < KC * NC && kg < kend && i < N) ? W[(pr.offC + kg) * N + i] : TC(0);
    }
  };
  auto store_w = [&](int buf, const TC (&src)[QW]) {
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < KC * NC) Ws[buf][e / NC][e % NC] = src[q];
    }
  };
  // Two register sets take turns (loop unrolled by two), so no copy forces
  // the prefetch to land early; W is loaded before A so that waiting for W
  // (to stage it in LDS) leaves the A loads in flight.
  TA a0[RT][KC / 4], a1[RT][KC / 4];
  TC wr[QW];
  load_w(kbeg, wr);
  load_a(kbeg, a0);
  store_w(0, wr);
  __syncthreads();
#define TIK_GN_STEP(CUR, NXT, KC0, BUF)                                                     \
  {                                                                                         \
    const bool more = (KC0) + KC < kend;                                                    \
    if (more) {                                                                             \
      load_w((KC0) + KC, wr);                                                               \
      load_a((KC0) + KC, NXT);                                                              \
    }                                                                                       \
    _Pragma("unroll") for (int ks = 0; ks < KC / 4; ++ks) {                                 \
      TC b[NT];                                                                             \
      _Pragma("unroll") for (int nt = 0; nt < NT; ++nt) b[nt] =                             \
          Ws[BUF][4 * ks + lk][nt * 16 + li];                                               \
      _Pragma("unroll") for (int rt = 0; rt < RT; ++rt)                                     \
          _Pragma("unroll") for (int nt = 0; nt < NT; ++nt) acc[rt][nt] =                   \
              M::op(TC(CUR[rt][ks]), b[nt], acc[rt][nt]);                                   \
    }                                                                                       \
    if (more) store_w((BUF) ^ 1, wr);                                                       \
    __syncthreads();                                                                        \
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += 2 * KC) {
    TIK_GN_STEP(a0, a1, k0, 0)
    if (k0 + KC >= kend) break;
    TIK_GN_STEP(a1, a0, k0 + KC, 1)
  }
#undef TIK_GN_STEP
  double nsum[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    nsum[nt] = 0.0;
    const int lam = nt * 16 + li;
    const double uc = (ep0 && lam < N) ? sc[it.p * N + lam].ucoef : 0.0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + rt * 16 + M::row(lane, v);
        if (row < m && lam < N) {
          const int64_t idx = (pr.offR + row) * N + lam;
          if (ep0) {
            const TC nv = TC(acc[rt][nt][v] - TC(uc) * ut[idx]);
            ut[idx] = nv;
            nsum[nt] += double(nv) * double(nv);
          } else if (EPI == 1) {
            out[idx] = double(acc[rt][nt][v]);
          } else {
            (EPI == 3 ? part2 : ut)[(pr.pnOff + int64_t(it.ch) * m + row) * N + lam] = acc[rt][nt][v];
          }
        }
      }
  }
  if (!ep0) return;                       // uniform over the block
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    double v = nsum[nt];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lk == 0) nred[wv][nt * 16 + li] = v;
  }
  __syncthreads();
  if (threadIdx.x < N)
    pnN[(pr.pnN + it.blk) * N + threadIdx.x] = nred[0][threadIdx.x] + nred[1][threadIdx.x] +
                                               nred[2][threadIdx.x] + nred[3][threadIdx.x];
}

// ------------------------------------------------------------------ gemm_t --
// Block = CB columns x one row chunk; wave w owns CB / 4 columns (CB = 64 for
// tall problems, 128 for wide ones, whose U is re-read by every column block).
// A (32 rows x CB columns) and U (32 rows x NC) are staged through LDS, then
// read in MFMA operand order (A^T as the A-operand, U as the B-operand).
// Blocks are remapped so that consecutive items (the column blocks of one row
// chunk, which share U) run on the same XCD and share its L2.
template <typename TA, typename TC, typename TU, int NC, int CB>
__global__ void __launch_bounds__(256) k_gemm_t_mfma(const DevProb* __restrict__ P,
                                                     const Item* __restrict__ items, int nitems,
                                                     int N, const TU* __restrict__ U,
                                                     TC* __restrict__ part) {
  using M = Mfma<TC>;
  constexpr int NT = NC / 16;
  constexpr int CT = CB / 64, RS = 32, AP = RS + 4, UP = NC + 2;
  __shared__ TA As[CB][AP];   // A as stored, widened to TC as the MFMA reads it
  __shared__ TC Us[RS][UP];
  const int g = blockIdx.x;
  const int per = (nitems + 7) >> 3;
  const int L = (g & 7) * per + (g >> 3);
  if (L >= nitems) return;
  const Item it = items[L];
  const DevProb& pr = P[it.p];
  if (pr.live && *pr.live == 0) return;   // every solve of the plan has stopped
  const TA* __restrict__ A = static_cast<const TA*>(pr.A);
  const int64_t m = pr.m, n = pr.n, lda = pr.lda;
  const int64_t c0 = int64_t(it.blk) * CB;
  const int64_t rbeg = int64_t(it.ch) * pr.rchunk;
  const int64_t rend = min(m, rbeg + pr.rchunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  typename M::acc_t acc[CT][NT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[ct][nt] = typename M::acc_t{0, 0, 0, 0};
  // The next tile of A and U is fetched into registers while the matrix cores
  // consume the current tile from LDS.
  constexpr int QA = (RS * CB) / 256;
  constexpr int QU = (RS * NC + 255) / 256;
  TA ra[QA];          // A as stored, widened when staged
  TC ru[QU];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int rr = e % RS, cc = e / RS;
      const int64_t rg = r0 + rr, cg = c0 + cc;
      ra[q] = (rg < rend && cg < n) ? A[rg + cg * lda] : TA(0);
    }
#pragma unroll
    for (int q = 0; q < QU; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int rr = e / NC, i = e % NC;
      const int64_t rg = r0 + rr;
      ru[q] = (e < RS * NC && rg < rend && i < N) ? TC(U[(pr.offR + rg) * N + i]) : TC(0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[e / RS][e % RS] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < QU; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < RS * NC) Us[e / NC][e % NC] = ru[q];
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
      TC a[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) a[ct] = TC(As[wv * (16 * CT) + ct * 16 + li][4 * ks + lk]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const TC b = Us[4 * ks + lk][nt * 16 + li];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct][nt] = M::op(a[ct], b, acc[ct][nt]);
      }
    }
    __syncthreads();
    if (more) stash();
    __syncthreads();
  }
  TC* dst = part + (pr.ptOff + int64_t(it.ch) * n) * N;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t c = c0 + wv * (16 * CT) + ct * 16 + M::row(lane, v);
        const int lam = nt * 16 + li;
        if (c < n && lam < N) dst[c * N + lam] = acc[ct][nt][v];
      }
}

// --------------------------------------------------------------- launchers --
template <typename TA, typename TC, int RT>
static int gemm_n_rt(int nc, int epi, const DevProb* P, const Item* items, int nitems, int N,
                     const void* Wv, void* ut, double* out, const Scal* sc, double* pnN,
                     const DevProb* P2, void* part2, hipStream_t st) {
  const TC* W = static_cast<const TC*>(Wv);
  const dim3 g = dim3(unsigned(nitems)), b = dim3(256);
  TC* u = static_cast<TC*>(ut);
  TC* p2 = static_cast<TC*>(part2);
#define TIK_GN(NCV, EPIV)                                                                     \
  if (nc == NCV && epi == EPIV) {                                                            \
    hipLaunchKernelGGL((k_gemm_n_mfma<TA, TC, NCV, EPIV, RT>), g, b, 0, st, P, items, N, W, u, \
                       out, sc, pnN, P2, p2);                                                \
    TIK_LAUNCHED("k_gemm_n_mfma");                                                           \
    return TIK_OK;                                                                           \
  }
  TIK_GN(16, 0) TIK_GN(32, 0) TIK_GN(16, 1) TIK_GN(32, 1) TIK_GN(16, 2) TIK_GN(32, 2)
  if constexpr (RT == 2) {
    TIK_GN(16, 3) TIK_GN(32, 3)
  }
#undef TIK_GN
  set_error("internal: MFMA gemm_n needs 16 or 32 lambdas per pass");
  return TIK_EINVAL;
}

template <typename TA, typename TC>
static int gemm_n_nc(int rows, int nc, int epi, const DevProb* P, const Item* items, int nitems,
                     int N, const void* W, void* ut, double* out, const Scal* sc, double* pnN,
                     const DevProb* P2, void* part2, hipStream_t st) {
  if (rows == 128)
    return gemm_n_rt<TA, TC, 2>(nc, epi, P, items, nitems, N, W, ut, out, sc, pnN, P2, part2, st);
  if (rows == 256 && epi != 3)
    return gemm_n_rt<TA, TC, 4>(nc, epi, P, items, nitems, N, W, ut, out, sc, pnN, P2, part2, st);
  set_error("internal: MFMA gemm_n blocks are 128 or 256 rows (128 with the tail's pieces)");
  return TIK_EINVAL;
}

int launch_gemm_n_mfma(int ta_f32, int tc_f32, int nc, int epi, int rows, const DevProb* P,
                       const Item* items, int nitems, int N, const void* W, void* ut,
                       double* out, const Scal* sc, double* pnN, hipStream_t st,
                       const DevProb* P2, void* part2) {
  if (epi == 3 && (!P2 || !part2)) {
    set_error("internal: the combined A W launch needs the tail's descriptor and buffer");
    return TIK_EINVAL;
  }
  if (tc_f32) {
    if (!ta_f32) {
      set_error("internal: FP32 products need FP32 storage");
      return TIK_EINVAL;
    }
    return gemm_n_nc<float, float>(rows, nc, epi, P, items, nitems, N, W, ut, out, sc, pnN, P2, part2, st);
  }
  if (ta_f32)
    return gemm_n_nc<float, double>(rows, nc, epi, P, items, nitems, N, W, ut, out, sc, pnN, P2, part2, st);
  return gemm_n_nc<double, double>(rows, nc, epi, P, items, nitems, N, W, ut, out, sc, pnN, P2, part2, st);
}

// Blocks of the 128-row EPI 0 product resident at once on the current device
// (blocks per CU from the occupancy calculator times the CU count), cached per
// device and shape; 0 if unknown.
int gemm_n_resident(int ta_f32, int tc_f32, int nc) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(dev, ta_f32, tc_f32, nc);
  std::lock_guard<std::mutex> lk(mu);
  auto hit = cache.find(key);
  if (hit != cache.end()) return hit->second;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn;
  if (tc_f32)
    fn = nc == 32 ? reinterpret_cast<const void*>(&k_gemm_n_mfma<float, float, 32, 0, 2>)
                  : reinterpret_cast<const void*>(&k_gemm_n_mfma<float, float, 16, 0, 2>);
  else if (ta_f32)
    fn = nc == 32 ? reinterpret_cast<const void*>(&k_gemm_n_mfma<float, double, 32, 0, 2>)
                  : reinterpret_cast<const void*>(&k_gemm_n_mfma<float, double, 16, 0, 2>);
  else
    fn = nc == 32 ? reinterpret_cast<const void*>(&k_gemm_n_mfma<double, double, 32, 0, 2>)
                  : reinterpret_cast<const void*>(&k_gemm_n_mfma<double, double, 16, 0, 2>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess) per = 0;
  (void)hipGetLastError();
  cache[key] = per * cus;
  return per * cus;
}

template <typename TA, typename TC, typename TU>
static int gemm_t_nc(int cols, int nc, const DevProb* P, const Item* items, int nitems, int N,
                     const void* U, void* part, hipStream_t st) {
  const dim3 g = dim3(unsigned(((nitems + 7) / 8) * 8)), b = dim3(256);
  const TU* u = static_cast<const TU*>(U);
  TC* pt = static_cast<TC*>(part);
#define TIK_GT(NCV, CBV)                                                                       \
  if (nc == NCV && cols == CBV) {                                                             \
    hipLaunchKernelGGL((k_gemm_t_mfma<TA, TC, TU, NCV, CBV>), g, b, 0, st, P, items, nitems, N, \
                       u, pt);                                                                \
    TIK_LAUNCHED("k_gemm_t_mfma");                                                            \
    return TIK_OK;                                                                            \
  }
  TIK_GT(16, 64) TIK_GT(32, 64) TIK_GT(16, 128) TIK_GT(32, 128)
#undef TIK_GT
  set_error("internal: MFMA gemm_t needs 16 or 32 lambdas and 64 or 128 columns per block");
  return TIK_EINVAL;
}

// U in TC (LSQR vectors) or FP64 (u_f64 = 1: refinement residuals, TC = double).
int launch_gemm_t_mfma(int ta_f32, int tc_f32, int u_f64, int nc, int cols, const DevProb* P,
                       const Item* items, int nitems, int N, const void* U, void* part,
                       hipStream_t st) {
  if (tc_f32) {
    if (!ta_f32) {
      set_error("internal: FP32 products need FP32 storage");
      return TIK_EINVAL;
    }
    if (u_f64) return gemm_t_nc<float, float, double>(cols, nc, P, items, nitems, N, U, part, st);
    return gemm_t_nc<float, float, float>(cols, nc, P, items, nitems, N, U, part, st);
  }
  if (ta_f32) return gemm_t_nc<float, double, double>(cols, nc, P, items, nitems, N, U, part, st);
  return gemm_t_nc<double, double, double>(cols, nc, P, items, nitems, N, U, part, st);
}

}  // namespace tik
