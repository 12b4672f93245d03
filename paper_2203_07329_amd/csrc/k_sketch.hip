// Sketch kernels: Y = X A (tall) or Y^T = X^T A^T (wide), X never stored whole.
//
// Embeddings (Section 2.1.1 of Meier & Nakatsukasa):
//  * SRHT  X = sqrt(m'/s) S H D with D random signs, H the orthonormal Hadamard
//          matrix of order m' = 2^k >= m (A zero-padded), S a uniform s-subset
//          of rows.  Applied as an unnormalised fast Walsh-Hadamard transform
//          (entries +-1) scaled by 1/sqrt(s), which is the same matrix.
//  * Gauss X with i.i.d. N(0, 1/s) entries, so E[X^T X] = I as the embedding
//          definition of Section 1.3 requires.
//
// Randomness comes from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// a counter-based generator, so every random entry is a pure function of
// (seed, index) and does not depend on launch shapes.
#include "tik_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <type_traits>

namespace tik {

// ---------------------------------------------------------------- Philox ----
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

static constexpr uint32_t TAG_PERM = 0x5052504Du;   // row subset
static constexpr uint32_t TAG_SIGN = 0x5349474Eu;   // random signs D
static constexpr uint32_t TAG_GAUS = 0x47415553u;   // Gaussian entries
static constexpr uint32_t TAG_SPAR = 0x53504152u;   // sparse embedding rows and signs

__device__ __forceinline__ uint2 seed_key(uint64_t seed) {
  return make_uint2(uint32_t(seed), uint32_t(seed >> 32));
}

// Balanced Feistel network on 2h bits with Philox round functions
// (Luby-Rackoff), restricted to [0, 2^k) by cycle walking.  A bijection of
// [0, 2^k), so its first s values are s distinct rows.  Out-of-range values
// number at most 2^(2h) - 2^k <= 2^k, so the walk ends within 2^k steps.
__device__ uint32_t feistel_perm(uint32_t x, int k, uint2 key) {
  const int h = (k + 1) >> 1;
  const uint32_t mask = (1u << h) - 1u;
  const uint32_t lim = 1u << k;
  for (uint32_t walk = 0; walk <= lim; ++walk) {
    uint32_t L = x >> h, R = x & mask;
#pragma unroll 1
    for (uint32_t r = 0; r < 6; ++r) {
      const uint32_t f = philox4x32_10(make_uint4(R, r, TAG_PERM, uint32_t(k)), key).x & mask;
      const uint32_t nl = R;
      R = L ^ f;
      L = nl;
    }
    x = (L << h) | R;
    if (x < lim) return x;
  }
  return 0xFFFFFFFFu;
}

// One workgroup: draw the s sampled rows (the first s values of the Feistel
// permutation of [0, 2^k)), mark them in an LDS bitmap of 2^k bits, and write
// them in ascending order: each thread owns a contiguous range of the bitmap's
// words, a prefix count over the block gives the rank of its first row, and
// its set bits follow in order.  The start of every bucket of 2^bbits
// consecutive rows (the number of sampled rows below it) comes from the same
// counts.  Also writes the sign bits of D (m'/32 words).  k <= ROWS_KMAX.
static constexpr int ROWS_KMAX = 18;

__global__ void __launch_bounds__(1024) k_srht_rows(uint64_t seed, int k, int64_t s,
                                                    int32_t* __restrict__ rows,
                                                    int32_t* __restrict__ bstart, int bbits,
                                                    uint32_t* __restrict__ signs) {
  __shared__ uint32_t bits[1 << (ROWS_KMAX - 5)];
  __shared__ int32_t wsum[16];
  const uint2 key = seed_key(seed);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int words = k >= 5 ? 1 << (k - 5) : 1;
  const uint32_t lim = 1u << k;
  for (int w = tid; w < words; w += 1024) bits[w] = 0u;
  __syncthreads();
  for (int64_t i = tid; i < s; i += 1024) {
    const uint32_t x = k == 0 ? 0u : feistel_perm(uint32_t(i), k, key);
    if (x < lim) atomicOr(&bits[x >> 5], 1u << (x & 31u));
  }
  __syncthreads();
  const int wpt = (words + 1023) / 1024;
  const int w0 = min(words, tid * wpt), w1 = min(words, w0 + wpt);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  int inc = cnt;                               // inclusive count within the wave
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int rank = inc - cnt;                        // rows below this thread's first word
  for (int q = 0; q < wv; ++q) rank += wsum[q];
  const int64_t step = int64_t(1) << bbits;
  for (int w = w0; w < w1; ++w) {
    const uint32_t v0 = bits[w];
    const int64_t p0 = int64_t(w) << 5;
    for (int64_t pos = (p0 + step - 1) / step * step; pos < p0 + 32 && pos < int64_t(lim); pos += step)
      bstart[pos >> bbits] = rank + __popc(v0 & ((1u << uint32_t(pos - p0)) - 1u));
    for (uint32_t v = v0; v; v &= v - 1u) rows[rank++] = int32_t(p0 + __ffs(v) - 1);
  }
  if (tid == 0) bstart[1 << (k - bbits)] = int32_t(s);
  const int nwords = ((1 << k) + 31) >> 5;
  for (int w = tid; w < nwords; w += blockDim.x) {
    const uint4 v = philox4x32_10(make_uint4(uint32_t(w >> 2), 0u, TAG_SIGN, 0u), key);
    const uint32_t sel = w & 3;
    signs[w] = sel == 0 ? v.x : sel == 1 ? v.y : sel == 2 ? v.z : v.w;
  }
}

__device__ __forceinline__ bool neg_sign(const uint32_t* __restrict__ signs, int64_t r) {
  return (signs[r >> 5] >> (r & 31)) & 1u;
}

// In-LDS Walsh-Hadamard transform of buf[0 .. 2^bits), all threads of the
// block taking part, for bits >= 3 whose first three stages (h = 1, 2, 4)
// the caller has already applied: the stages commute, so the rest run as
// radix-8 passes (three stages on 8 values in registers per LDS round trip),
// then one radix-4 or radix-2 pass for the remainder.  Group g of a pass at
// stage t holds the elements i + j 2^t, i = g with three zero bits inserted at t.
__device__ __forceinline__ void fwht_lds_from3(double* buf, int bits) {
  const int M = 1 << bits;
  int t = 3;
  for (; t + 3 <= bits; t += 3) {
    const int h = 1 << t;
    for (int g = threadIdx.x; g < (M >> 3); g += blockDim.x) {
      const int i = ((g >> t) << (t + 3)) | (g & (h - 1));
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = buf[i + j * h];
#pragma unroll
      for (int hh = 1; hh < 8; hh <<= 1)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if ((j & hh) == 0) {
            const double a = v[j], b = v[j + hh];
            v[j] = a + b;
            v[j + hh] = a - b;
          }
#pragma unroll
      for (int j = 0; j < 8; ++j) buf[i + j * h] = v[j];
    }
    __syncthreads();
  }
  const int r = bits - t;
  if (r == 2) {
    const int h = 1 << t;
    for (int g = threadIdx.x; g < (M >> 2); g += blockDim.x) {
      const int i = ((g >> t) << (t + 2)) | (g & (h - 1));
      double v0 = buf[i], v1 = buf[i + h], v2 = buf[i + 2 * h], v3 = buf[i + 3 * h];
      const double a0 = v0 + v1, a1 = v0 - v1, a2 = v2 + v3, a3 = v2 - v3;
      buf[i] = a0 + a2;
      buf[i + h] = a1 + a3;
      buf[i + 2 * h] = a0 - a2;
      buf[i + 3 * h] = a1 - a3;
    }
    __syncthreads();
  } else if (r == 1) {
    const int h = 1 << t;
    for (int g = threadIdx.x; g < (M >> 1); g += blockDim.x) {
      const int i = ((g >> t) << (t + 1)) | (g & (h - 1));
      const double a = buf[i], b = buf[i + h];
      buf[i] = a + b;
      buf[i + h] = a - b;
    }
    __syncthreads();
  }
}

// Stages h = 1, 2, 4 on 8 consecutive values in registers.
__device__ __forceinline__ void fwht8(double (&v)[8]) {
#pragma unroll
  for (int hh = 1; hh < 8; hh <<= 1)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if ((j & hh) == 0) {
        const double a = v[j], b = v[j + hh];
        v[j] = a + b;
        v[j + hh] = a - b;
      }
}

// Single-pass SRHT for m' <= 2^13: one workgroup per column, the whole padded
// column staged in LDS, log2 m' butterfly stages, then the sampled rows gathered.
template <typename TA>
__global__ void __launch_bounds__(256) k_srht_single(const TA* __restrict__ A, int64_t m,
                                                     int64_t lda, int k,
                                                     const uint32_t* __restrict__ signs,
                                                     const int32_t* __restrict__ rows, int64_t s,
                                                     double scale, double* __restrict__ Y) {
  extern __shared__ double lbuf[];
  const int64_t c = blockIdx.x;
  const int M = 1 << k;
  const TA* col = A + c * lda;
  if (k >= 3) {
    for (int g = threadIdx.x; g < (M >> 3); g += blockDim.x) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t r = 8 * int64_t(g) + j;
        double x = 0.0;
        if (r < m) {
          x = double(col[r]);
          if (neg_sign(signs, r)) x = -x;
        }
        v[j] = x;
      }
      fwht8(v);
#pragma unroll
      for (int j = 0; j < 8; ++j) lbuf[8 * g + j] = v[j];
    }
    __syncthreads();
    fwht_lds_from3(lbuf, k);
  } else {
    for (int r = threadIdx.x; r < M; r += blockDim.x) {
      double v = 0.0;
      if (r < m) {
        v = double(col[r]);
        if (neg_sign(signs, r)) v = -v;
      }
      lbuf[r] = v;
    }
    __syncthreads();
    for (int h = 1; h < M; h <<= 1) {
      for (int idx = threadIdx.x; idx < (M >> 1); idx += blockDim.x) {
        const int i = ((idx & ~(h - 1)) << 1) | (idx & (h - 1));
        const double a = lbuf[i], b = lbuf[i + h];
        lbuf[i] = a + b;
        lbuf[i + h] = a - b;
      }
      __syncthreads();
    }
  }
  for (int64_t q = threadIdx.x; q < s; q += blockDim.x) Y[q + c * s] = lbuf[rows[q]] * scale;
}

// Two-pass SRHT, H_{2^k} = H_{2^a} (x) H_{2^b} with k = a + b.
// Pass 1 applies H_{2^a} across the 2^a rows hi*2^b + lo sharing a low index
// (one thread per lo, 2^a values in registers; threads read consecutive rows).
template <typename TA, int ABITS>
__global__ void __launch_bounds__(256) k_srht_pass1(const TA* __restrict__ A, int64_t m,
                                                    int64_t lda, int64_t c0, int bbits,
                                                    const uint32_t* __restrict__ signs,
                                                    double* __restrict__ T) {
  constexpr int NA = 1 << ABITS;
  const int64_t lo = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t cc = blockIdx.y;
  const int64_t B = int64_t(1) << bbits;
  if (lo >= B) return;
  const TA* col = A + (c0 + cc) * lda;
  double v[NA];
#pragma unroll
  for (int hi = 0; hi < NA; ++hi) {
    const int64_t r = hi * B + lo;
    double x = 0.0;
    if (r < m) {
      x = double(col[r]);
      if (neg_sign(signs, r)) x = -x;
    }
    v[hi] = x;
  }
#pragma unroll
  for (int h = 1; h < NA; h <<= 1) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if ((i & h) == 0) {
        const double a = v[i], b = v[i + h];
        v[i] = a + b;
        v[i + h] = a - b;
      }
    }
  }
  double* tcol = T + cc * (B << ABITS);
#pragma unroll
  for (int hi = 0; hi < NA; ++hi) tcol[hi * B + lo] = v[hi];
}

// Pass 2 applies H_{2^b} to each contiguous bucket of 2^b rows in LDS and
// writes only the sampled rows that fall in the bucket.
__global__ void __launch_bounds__(256) k_srht_pass2(const double* __restrict__ T, int64_t c0,
                                                    int k, int bbits,
                                                    const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ bstart, int64_t s,
                                                    double scale, double* __restrict__ Y) {
  extern __shared__ double lbuf[];
  const int hb = blockIdx.x;
  const int64_t cc = blockIdx.y;
  const int B = 1 << bbits;
  const int q0 = bstart[hb], q1 = bstart[hb + 1];
  if (q0 == q1) return;
  const double* src = T + cc * (int64_t(1) << k) + int64_t(hb) * B;
  if (bbits >= 3) {
    for (int g = threadIdx.x; g < (B >> 3); g += blockDim.x) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = src[8 * g + j];
      fwht8(v);
#pragma unroll
      for (int j = 0; j < 8; ++j) lbuf[8 * g + j] = v[j];
    }
    __syncthreads();
    fwht_lds_from3(lbuf, bbits);
  } else {
    for (int r = threadIdx.x; r < B; r += blockDim.x) lbuf[r] = src[r];
    __syncthreads();
    for (int h = 1; h < B; h <<= 1) {
      for (int idx = threadIdx.x; idx < (B >> 1); idx += blockDim.x) {
        const int i = ((idx & ~(h - 1)) << 1) | (idx & (h - 1));
        const double a = lbuf[i], b = lbuf[i + h];
        lbuf[i] = a + b;
        lbuf[i + h] = a - b;
      }
      __syncthreads();
    }
  }
  const int64_t base = int64_t(hb) * B;
  for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x)
    Y[q + (c0 + cc) * s] = lbuf[rows[q] - base] * scale;
}

// Column-resident SRHT for m' = 2^k >= 2^14: one 512-thread workgroup per
// column (the bucket fills most of a CU's LDS, so one workgroup per CU).
// Writing a row index as r = hi 2^14 + lo, H_{2^k} = H_{2^(k-14)} (x) H_{2^14},
// so entry (ihi, ilo) of H D a is the sum over buckets hi of
// (-1)^popcount(ihi & hi) times entry ilo of H_{2^14} applied to bucket hi.
// Each bucket of 2^14 rows is transformed in LDS in three register phases (32
// entries per thread: five, five and four butterfly stages) and every sampled
// row adds its entry with its sign, so A is read from HBM once and only Y is
// written.  Buckets wholly beyond row m are zero and skipped.  Loading the next
// bucket into registers while the current one is transformed was measured
// slower (1.45 against 1.08 ms for the 200000 x 2000 sketch with s = 8000: the
// extra 64 registers spill), as were buckets of 2^13 rows with two workgroups
// per CU (1.85 ms: 32 sampled rows per thread spill).
static constexpr int SRC_BITS = 14;
static constexpr int SRC_T = 1 << (SRC_BITS - 5);
// two doubles of padding per 32 entries: a thread's run of 32 consecutive
// entries starts 34 doubles after its neighbour's, four banks further on
__device__ __forceinline__ int src_pad(int x) { return x + 2 * (x >> 5); }

// butterfly stages of v over the low NB bits of the register index
template <int NB>
__device__ __forceinline__ void fwht32_low(double (&v)[32]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int hh = 1 << b;
#pragma unroll
    for (int j = 0; j < 32; ++j)
      if ((j & hh) == 0) {
        const double a = v[j], c = v[j + hh];
        v[j] = a + c;
        v[j + hh] = a - c;
      }
  }
}

template <typename TA, int QV>
__global__ void __launch_bounds__(SRC_T) k_srht_cols(const TA* __restrict__ A, int64_t m,
                                                     int64_t lda,
                                                     const uint32_t* __restrict__ signs,
                                                     const int32_t* __restrict__ rows, int64_t s,
                                                     double scale, double* __restrict__ Y) {
  constexpr int BITS = SRC_BITS;
  constexpr int B = 1 << BITS;
  constexpr int T = SRC_T;   // threads, and sign words per bucket
  __shared__ double lb[B + B / 16];
  __shared__ uint32_t sg[2][T];
  const int t = threadIdx.x;
  const TA* col = A + int64_t(blockIdx.x) * lda;
  const int m32 = int(m);
  const int nbk = (m32 + B - 1) >> BITS;
  // sampled row q = t + T u: its padded LDS position within a bucket in the
  // low 15 bits, its bucket index ihi above them (-1: no such row)
  int32_t gq[QV];
  double acc[QV];
#pragma unroll
  for (int u = 0; u < QV; ++u) {
    const int64_t q = t + int64_t(T) * u;
    const int32_t r = q < s ? rows[q] : -1;
    gq[u] = r < 0 ? -1 : ((r >> BITS) << 15) | src_pad(r & (B - 1));
    acc[u] = 0.0;
  }
  // phase 1: register j holds lo = T j + t (coalesced).  Buffer loads through a
  // resource based at the bucket's first row and bounded at row m, with the
  // whole offset in the VGPR: entries past row m lie outside the resource and
  // read as zero (the select zeroes them again).
  TA raw[32];
  auto load = [&](int hi) {
    const int r0 = hi << BITS;
    const int nrec = m32 - r0;
    // stride 0 (raw buffer), size in bytes, and the gfx9 word 3 for untyped
    // dword access
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TA*>(col + r0), 0, nrec * int(sizeof(TA)), 0x00020000);
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const int lo = j * T + t;
      TA x;
      if constexpr (sizeof(TA) == 8)
        x = __builtin_bit_cast(TA, __builtin_amdgcn_raw_buffer_load_b64(rs, lo * 8, 0, 0));
      else
        x = __builtin_bit_cast(TA, __builtin_amdgcn_raw_buffer_load_b32(rs, lo * 4, 0, 0));
      raw[j] = lo < nrec ? x : TA(0);
    }
  };
  sg[0][t] = signs[t];
  __syncthreads();
  // LDS positions as a per-thread base plus a constant per register
  const int b1 = t + 2 * (t >> 5);                       // src_pad(T j + t) = b1 + (17 T / 16) j
  const int b2 = 34 * t;                                 // src_pad(32 t + j) = b2 + j
  const int b3 = src_pad((t & 31) | ((t >> 5) << 10));   // src_pad(lo3 | 32 j) = b3 + 34 j
  // one bucket; with `more` the next bucket's sign words are staged (the last
  // bucket is peeled off below)
  auto bucket = [&](int hi, auto more_tag) {
    constexpr bool more = decltype(more_tag)::value;
    load(hi);
    const uint32_t* sgc = sg[hi & 1];
    double v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const double x = double(raw[j]);
      v[j] = ((sgc[j * (T / 32) + (t >> 5)] >> (t & 31)) & 1u) ? -x : x;
    }
    // the next bucket's sign word, staged in LDS before the gather
    uint32_t snext = 0;
    if (more) snext = signs[int64_t(hi + 1) * T + t];
    fwht32_low<5>(v);  // lo bits BITS-5 .. BITS-1
    __syncthreads();   // every thread has gathered from the previous bucket
#pragma unroll
    for (int j = 0; j < 32; ++j) lb[b1 + (17 * T / 16) * j] = v[j];
    __syncthreads();
    // phase 2: thread t holds lo = 32 t + j
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = lb[b2 + j];
    fwht32_low<5>(v);  // lo bits 0..4
#pragma unroll
    for (int j = 0; j < 32; ++j) lb[b2 + j] = v[j];
    __syncthreads();
    // phase 3: lo bits 0..4 from t % 32, 5..9 from j, 10.. from t / 32; the
    // bits from BITS - 5 on were done in phase 1
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = lb[b3 + 34 * j];
    fwht32_low<BITS - 10>(v);  // lo bits 5 .. BITS-6
#pragma unroll
    for (int j = 0; j < 32; ++j) lb[b3 + 34 * j] = v[j];
    if (more) sg[(hi + 1) & 1][t] = snext;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < QV; ++u)
      if (gq[u] >= 0) {
        const double z = lb[gq[u] & 0x7FFF];
        acc[u] += (__popc(uint32_t(gq[u] >> 15) & uint32_t(hi)) & 1) ? -z : z;
      }
  };
  for (int hi = 0; hi + 1 < nbk; ++hi) bucket(hi, std::true_type{});
  bucket(nbk - 1, std::false_type{});
#pragma unroll
  for (int u = 0; u < QV; ++u) {
    const int64_t q = t + int64_t(T) * u;
    if (q < s) Y[q + int64_t(blockIdx.x) * s] = acc[u] * scale;
  }
}

// ---------------------------------------------------------------- Gaussian --
// Entry (q, r) of the s x (long dim) Gaussian matrix: Philox of counter
// (r, q/4) gives four 32-bit words, Box-Muller turns them into four normals
// for rows q = 4*(q/4) .. +3.  Scaled by 1/sqrt(s).
__device__ __forceinline__ void gauss4(uint64_t seed, uint32_t r, uint32_t qb, double out[4]) {
  const uint4 v = philox4x32_10(make_uint4(r, qb, TAG_GAUS, 0u), seed_key(seed));
  const double two32 = 4294967296.0;
  const double u0 = (double(v.x) + 0.5) / two32, u1 = (double(v.y) + 0.5) / two32;
  const double u2 = (double(v.z) + 0.5) / two32, u3 = (double(v.w) + 0.5) / two32;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double s0, c0, s1, c1;
  sincospi(2.0 * u1, &s0, &c0);
  sincospi(2.0 * u3, &s1, &c1);
  out[0] = r0 * c0;
  out[1] = r0 * s0;
  out[2] = r1 * c1;
  out[3] = r1 * s1;
}

// X chunk (s x kc, column-major ld = s): columns are long-dimension indices
// r0 .. r0 + kc - 1.  One thread per (4 rows, 1 column).
template <typename TX>
__global__ void __launch_bounds__(256) k_gauss_gen(uint64_t seed, int64_t s, int64_t r0,
                                                   int64_t kc, double scale, TX* __restrict__ X) {
  const int64_t sq = (s + 3) >> 2;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= sq * kc) return;
  const int64_t qb = idx % sq, cc = idx / sq;
  double z[4];
  gauss4(seed, uint32_t(r0 + cc), uint32_t(qb), z);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t q = qb * 4 + t;
    if (q < s) X[q + cc * s] = TX(z[t] * scale);
  }
}

// Y (s x ncol, ld = s) += Xc (s x kc, ld = s) * Bop (kc x ncol), FP64,
// Bop(kk, c) = A[(r0 + kk) + c lda] (tall) or A[c + (r0 + kk) lda] (wide).
// 64 x 64 output tile, 16-deep k steps staged in LDS, 4 x 4 per thread.
template <typename TA, bool WIDE>
__global__ void __launch_bounds__(256) k_sketch_gemm64(const double* __restrict__ Xc, int64_t s,
                                                       int64_t kc, const TA* __restrict__ A,
                                                       int64_t lda, int64_t r0, int64_t ncol,
                                                       double* __restrict__ Y) {
  __shared__ double Xs[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int64_t q0 = int64_t(blockIdx.x) * 64, c0 = int64_t(blockIdx.y) * 64;
  const int tq = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < kc; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int qq = e & 63, kk = e >> 6;
      const int64_t q = q0 + qq, kg = k0 + kk;
      Xs[kk][qq] = (q < s && kg < kc) ? Xc[q + kg * s] : 0.0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      int kk, cc;
      if (WIDE) { cc = e & 63; kk = e >> 6; } else { kk = e & 15; cc = e >> 4; }
      const int64_t c = c0 + cc, kg = k0 + kk;
      double v = 0.0;
      if (c < ncol && kg < kc) v = WIDE ? double(A[c + (r0 + kg) * lda]) : double(A[(r0 + kg) + c * lda]);
      Bs[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double xa[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = Xs[kk][tq + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(xa[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t q = q0 + tq + 16 * i, c = c0 + tc + 16 * j;
      if (q < s && c < ncol) Y[q + c * s] += acc[i][j];
    }
}

// ------------------------------------------------------------ BF16 sketch --
// The four normals of gauss4 from the same Philox counters, Box-Muller in
// FP32 but with every quantity an FP32 relative error away from the exact one,
// so that the BF16-rounded entries agree with the rounded FP64 ones:
//   ln u = log((x + 1/2) 2^-32) for x < 2^31, else log1p(-(2^32 - x - 1/2) 2^-32)
//     (1 - u is formed from the integer, exact);
//   the angle 2 pi u' is reduced to a quadrant on the integer, and both its
//   sine and cosine are sinpi of an offset formed exactly from the integer.
__device__ __forceinline__ float lr_log_u(uint32_t x) {
  const float inv32 = 2.3283064365386963e-10f;   // 2^-32
  if (x < 0x80000000u) return logf((float(x) + 0.5f) * inv32);
  return log1pf(-(float(0xFFFFFFFFu - x) + 0.5f) * inv32);
}
__device__ __forceinline__ void lr_sincos_2pi_u(uint32_t y, float& sn, float& cs) {
  const uint32_t q = y >> 30, f = y & 0x3FFFFFFFu;   // quadrant, offset within it
  const float inv31 = 4.656612873077393e-10f;      // 2^-31
  const float a = sinpif((float(f) + 0.5f) * inv31);               // sin of the offset angle
  const float b = sinpif((float(0x3FFFFFFFu - f) + 0.5f) * inv31); // its cosine
  switch (q) {
    case 0: sn = a; cs = b; break;
    case 1: sn = b; cs = -a; break;
    case 2: sn = -a; cs = -b; break;
    default: sn = -b; cs = a; break;
  }
}
__device__ __forceinline__ void gauss4f(uint64_t seed, uint32_t r, uint32_t qb, float out[4]) {
  const uint4 v = philox4x32_10(make_uint4(r, qb, TAG_GAUS, 0u), seed_key(seed));
  const float r0 = sqrtf(-2.0f * lr_log_u(v.x)), r1 = sqrtf(-2.0f * lr_log_u(v.z));
  float s0, c0, s1, c1;
  lr_sincos_2pi_u(v.y, s0, c0);
  lr_sincos_2pi_u(v.w, s1, c1);
  out[0] = r0 * c0;
  out[1] = r0 * s0;
  out[2] = r1 * c1;
  out[3] = r1 * s1;
}

// X chunk in BF16 or FP16, stored row-major s x kc (k contiguous), the layout
// the matrix-core operand loads want: the Philox/Box-Muller normals of the
// FP64 generator (computed in FP32, see gauss4f), rounded to the 16-bit type.
__device__ __forceinline__ uint16_t to16(float v, __hip_bfloat16*) {
  const __hip_bfloat16 h = __float2bfloat16(v);
  return *reinterpret_cast<const uint16_t*>(&h);
}
__device__ __forceinline__ uint16_t to16(float v, _Float16*) {
  const _Float16 h = static_cast<_Float16>(v);    // round to nearest even
  return *reinterpret_cast<const uint16_t*>(&h);
}
template <typename T16>
__device__ __forceinline__ void gauss_gen16(uint64_t seed, int64_t s, int64_t r0, int64_t kc, int64_t ldx,
                                            float scale, uint16_t* __restrict__ X) {
  const int64_t sq = (s + 3) >> 2;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= sq * kc) return;
  const int64_t cc = idx % kc, qb = idx / kc;
  float z[4];
  gauss4f(seed, uint32_t(r0 + cc), uint32_t(qb), z);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t q = qb * 4 + t;
    if (q < s) X[q * ldx + cc] = to16(z[t] * scale, static_cast<T16*>(nullptr));
  }
}
__global__ void __launch_bounds__(256) k_gauss_gen_bf16(uint64_t seed, int64_t s, int64_t r0,
                                                        int64_t kc, int64_t ldx, float scale,
                                                        __hip_bfloat16* __restrict__ X) {
  gauss_gen16<__hip_bfloat16>(seed, s, r0, kc, ldx, scale, reinterpret_cast<uint16_t*>(X));
}
__global__ void __launch_bounds__(256) k_gauss_gen_f16(uint64_t seed, int64_t s, int64_t r0,
                                                       int64_t kc, int64_t ldx, float scale,
                                                       _Float16* __restrict__ X) {
  gauss_gen16<_Float16>(seed, s, r0, kc, ldx, scale, reinterpret_cast<uint16_t*>(X));
}

typedef __bf16 sk_bf16x8 __attribute__((ext_vector_type(8)));

// 16 consecutive values from a 16-byte-aligned address, as 16-byte loads.
__device__ __forceinline__ void lr16(const float* src, float (&d)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = reinterpret_cast<const float4*>(src)[q];
    d[4 * q] = v.x;
    d[4 * q + 1] = v.y;
    d[4 * q + 2] = v.z;
    d[4 * q + 3] = v.w;
  }
}
__device__ __forceinline__ void lr4(const float* src, float* d) {
  const float4 v = *reinterpret_cast<const float4*>(src);
  d[0] = v.x;
  d[1] = v.y;
  d[2] = v.z;
  d[3] = v.w;
}
__device__ __forceinline__ void lr4(const double* src, float* d) {
  const double2 v0 = reinterpret_cast<const double2*>(src)[0];
  const double2 v1 = reinterpret_cast<const double2*>(src)[1];
  d[0] = float(v0.x);
  d[1] = float(v0.y);
  d[2] = float(v1.x);
  d[3] = float(v1.y);
}
__device__ __forceinline__ void lr16(const double* src, float (&d)[16]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double2 v = reinterpret_cast<const double2*>(src)[q];
    d[2 * q] = float(v.x);
    d[2 * q + 1] = float(v.y);
  }
}
typedef float sk_f32x16 __attribute__((ext_vector_type(16)));

template <typename T16>
__device__ __forceinline__ uint32_t pack16(float a, float b) {
  return uint32_t(to16(a, static_cast<T16*>(nullptr))) | (uint32_t(to16(b, static_cast<T16*>(nullptr))) << 16);
}
typedef _Float16 sk_f16x8 __attribute__((ext_vector_type(8)));

// Yacc (s x ncol, ld s, FP32) (+)= X (s x kc, BF16, ld kc) * Bop (kc x ncol), Bop(k, c) =
// A[(r0 + k) + c lda] (tall) or A[c + (r0 + k) lda] (wide), rounded to BF16.
// ST x 128 output tile per block (ST = 128 or 256 rows of the sketch), 4 waves
// of ST/2 x 64 (ST/64 x 2 tiles of v_mfma_f32_32x32x16_bf16: A-operand lane l holds row l % 32, k = 8 (l / 32) .. +7;
// B-operand lane l holds column l % 32 at the same k; the 16 results of lane l
// are rows 8 (v / 4) + 4 (l / 32) + v % 4 of column l % 32).  Tiles of KB k are
// staged in LDS k-contiguous (row / column major) so each operand is one
// 16-byte read; LDS holds two stages, so the next step (fetched into
// registers with 16-byte loads during the MFMAs) is written to the other stage
// and one barrier per step suffices.  ST = 256 halves the A tile loads per
// flop (each step's A tile serves twice the sketch rows).
// Split K (grid.z > 1): block z covers k in [z ksz, (z + 1) ksz) and stores its
// partial product to Y + z s ncol; k_sketch_reduce adds the slices in order.
// Tile placement: workgroups are dealt to the 8 XCDs in turn (block g runs on
// XCD g mod 8), so XCD x gets the rectangle (x / pc, x mod pc) of a ps x pc
// split of the tile grid (sR x cR tiles each), walked row by row: the
// workgroups running together on one XCD share their X rows and A columns in
// that XCD's L2, and each operand panel is fetched by ps or pc XCDs only.
template <typename T16, typename TA, bool WIDE, int KB, int ST>
__device__ __forceinline__ void sketch_gemm_body(const uint16_t* __restrict__ X, int64_t s, int64_t kc,
                                                 int64_t ldx, int64_t ksz, const TA* __restrict__ A,
                                                 int64_t lda, int64_t r0, int64_t ncol, int sR, int cR,
                                                 int pc, float* __restrict__ Y, int first,
                                                 const float* __restrict__ cscale) {
  static_assert(KB % 32 == 0 && KB <= 128, "k per step");
  static_assert(ST == 128 || ST == 256, "sketch rows per tile");
  constexpr int LP = KB + 8;              // LDS row pitch in bf16
  constexpr int HK = KB / 2;              // k per thread (tall B): half a row of the step
  constexpr int TPR = 256 / ST;           // threads per X row
  constexpr int XK = KB / TPR;            // k per thread (X)
  constexpr int AT = ST / 64;             // 32-row MFMA tiles per wave
  constexpr int WK = KB / 8;              // k per thread (wide B)
  const int xcd = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int64_t stile = int64_t(xcd / pc) * sR + jx / cR, ctile = int64_t(xcd % pc) * cR + jx % cR;
  if (jx >= sR * cR || stile * ST >= s || ctile * 128 >= ncol) return;   // uniform
  const int64_t kb = int64_t(blockIdx.z) * ksz, ke = min(kc, kb + ksz);
  if (gridDim.z > 1) {
    Y += int64_t(blockIdx.z) * s * ncol;
    first = 1;
  }
  __shared__ __attribute__((aligned(16))) uint16_t Xs2[2][ST * LP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs2[2][128 * LP];
  uint16_t* Xs = Xs2[0];
  uint16_t* Bs = Bs2[0];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wq = wv >> 1, wc = wv & 1;
  const int64_t q0 = stile * ST, c0 = ctile * 128;
  sk_f32x16 acc[AT][2];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;
  // register stage of one step: X (XK bf16 per thread), B (HK values per thread).
  // Every whole step is prefetched during the previous step's MFMAs: X rows
  // (pitch ldx, a multiple of 8) with 16-byte loads, A with 16-byte loads
  // where its runs start 16-byte aligned (base, lda and the chunk origin
  // multiples of 16 bytes / sizeof(TA)), else with one load per element (a
  // tall A whose row count is odd, say).  The ragged last step is copied
  // element by element into LDS after the barrier.
  uint4 rx[XK / 8];
  float rb[HK];
  constexpr int64_t VE = 16 / sizeof(TA);
  const bool vx = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && (ldx & 7) == 0;
  const bool va = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && lda % VE == 0 && r0 % VE == 0 &&
                  (WIDE ? (c0 % VE == 0) : (kb % VE == 0));
  auto whole = [&](int64_t k0) { return vx && k0 + KB <= ke; };
  auto fetch = [&](int64_t k0) {               // whole steps only
    {
      const int row = tid / TPR, part = tid % TPR;
      const int64_t q = q0 + row;
#pragma unroll
      for (int h = 0; h < XK / 8; ++h)
        rx[h] = q < s ? *reinterpret_cast<const uint4*>(X + q * ldx + k0 + part * XK + h * 8)
                      : make_uint4(0, 0, 0, 0);
    }
    if (!WIDE) {
      const int col = tid >> 1, half = tid & 1;
      const int64_t c = c0 + col;
      const TA* src = A + (r0 + k0 + half * HK) + min(c, ncol - 1) * lda;
      if (va) {
#pragma unroll
        for (int h = 0; h < HK / 16; ++h) lr16(src + 16 * h, *reinterpret_cast<float(*)[16]>(rb + 16 * h));
      } else {
#pragma unroll
        for (int e = 0; e < HK; ++e) rb[e] = float(src[e]);
      }
      if (c >= ncol)
#pragma unroll
        for (int e = 0; e < HK; ++e) rb[e] = 0.f;
    } else {
      // 4 consecutive rows of A (operand columns c, contiguous) at each of WK
      // consecutive k: rb[4 kk + j] = element (k = WK k4 + kk, c = 4 c4 + j)
      const int c4 = tid & 31, k4 = tid >> 5;
      const int64_t c = c0 + 4 * c4;
      const bool cin = c + 4 <= ncol;
#pragma unroll
      for (int kk = 0; kk < WK; ++kk) {
        const int64_t k = k0 + WK * k4 + kk;
        if (cin && va) {
          lr4(A + c + (r0 + k) * lda, rb + 4 * kk);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            rb[4 * kk + j] = c + j < ncol ? float(A[(c + j) + (r0 + k) * lda]) : 0.f;
        }
      }
    }
  };
  auto stash = [&]() {                          // the fetched whole step
    {
      const int row = tid / TPR, part = tid % TPR;
#pragma unroll
      for (int h = 0; h < XK / 8; ++h)
        *reinterpret_cast<uint4*>(&Xs[row * LP + part * XK + 8 * h]) = rx[h];
    }
    if (!WIDE) {
      const int col = tid >> 1, half = tid & 1;
      // the column's power-of-two scale (FP16 operands), exact
      const float sc = cscale ? cscale[min(c0 + col, ncol - 1)] : 1.f;
#pragma unroll
      for (int h = 0; h < HK / 8; ++h)
        *reinterpret_cast<uint4*>(&Bs[col * LP + half * HK + 8 * h]) =
            make_uint4(pack16<T16>(sc * rb[8 * h], sc * rb[8 * h + 1]), pack16<T16>(sc * rb[8 * h + 2], sc * rb[8 * h + 3]),
                       pack16<T16>(sc * rb[8 * h + 4], sc * rb[8 * h + 5]), pack16<T16>(sc * rb[8 * h + 6], sc * rb[8 * h + 7]));
    } else {
      // column 4 c4 + j gets its WK k values, 8 bytes (4 k) per write
      const int c4 = tid & 31, k4 = tid >> 5;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int g = 0; g < WK / 4; ++g)
          *reinterpret_cast<uint2*>(&Bs[(4 * c4 + j) * LP + WK * k4 + 4 * g]) =
              make_uint2(pack16<T16>(rb[4 * (4 * g) + j], rb[4 * (4 * g + 1) + j]),
                         pack16<T16>(rb[4 * (4 * g + 2) + j], rb[4 * (4 * g + 3) + j]));
    }
  };
  auto stash_ragged = [&](int64_t k0) {         // element by element, zeros outside
    for (int e = tid; e < ST * KB; e += 256) {
      const int r = e / KB, kk = e % KB;
      const int64_t k = k0 + kk, q = q0 + r;
      Xs[r * LP + kk] = (q < s && k < ke) ? X[q * ldx + k] : 0;
    }
    for (int e = tid; e < 128 * KB; e += 256) {
      const int r = e / KB, kk = e % KB;
      const int64_t k = k0 + kk, c = c0 + r;
      const float v = (c < ncol && k < ke) ? float(WIDE ? A[c + (r0 + k) * lda] : A[(r0 + k) + c * lda])
                                           : 0.f;
      const float sc = (cscale && c < ncol) ? cscale[c] : 1.f;
      Bs[r * LP + kk] = to16(sc * v, static_cast<T16*>(nullptr));
    }
  };
  if (whole(kb)) {
    fetch(kb);
    stash();
  } else {
    stash_ragged(kb);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += KB) {
    const bool more = k0 + KB < ke, pre = more && whole(k0 + KB);
    if (pre) fetch(k0 + KB);
    Xs = Xs2[buf];
    Bs = Bs2[buf];
#pragma unroll
    for (int ks = 0; ks < KB / 16; ++ks) {
      uint4 av[AT], bv[2];
      const int kofs = ks * 16 + 8 * (lane >> 5);
#pragma unroll
      for (int t = 0; t < AT; ++t) {
        const int row = wq * (ST / 2) + t * 32 + (lane & 31);
        av[t] = *reinterpret_cast<const uint4*>(&Xs[row * LP + kofs]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = wc * 64 + t * 32 + (lane & 31);
        bv[t] = *reinterpret_cast<const uint4*>(&Bs[col * LP + kofs]);
      }
#pragma unroll
      for (int a = 0; a < AT; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if constexpr (std::is_same<T16, _Float16>::value)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(sk_f16x8, av[a]),
                                                               __builtin_bit_cast(sk_f16x8, bv[b]), acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(sk_bf16x8, av[a]),
                                                                __builtin_bit_cast(sk_bf16x8, bv[b]), acc[a][b], 0, 0, 0);
        }
    }
    // the next step goes to the other stage: one barrier per step
    Xs = Xs2[buf ^ 1];
    Bs = Bs2[buf ^ 1];
    if (pre) stash();
    else if (more) stash_ragged(k0 + KB);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t q = q0 + wq * (ST / 2) + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t c = c0 + wc * 64 + b * 32 + (lane & 31);
        if (q < s && c < ncol) {
          float* dst = Y + q + c * s;
          *dst = first ? acc[a][b][v] : *dst + acc[a][b][v];
        }
      }
}


template <typename TA, bool WIDE, int KB, int ST>
__global__ void __launch_bounds__(256, ST == 256 ? 2 : 1) k_sketch_gemm_bf16(const __hip_bfloat16* __restrict__ X,
                                                          int64_t s, int64_t kc, int64_t ldx,
                                                          int64_t ksz,
                                                          const TA* __restrict__ A, int64_t lda,
                                                          int64_t r0, int64_t ncol, int sR, int cR,
                                                          int pc, float* __restrict__ Y, int first) {
  sketch_gemm_body<__hip_bfloat16, TA, WIDE, KB, ST>(reinterpret_cast<const uint16_t*>(X), s, kc, ldx, ksz, A,
                                                     lda, r0, ncol, sR, cR, pc, Y, first, nullptr);
}

// The FP16 product of a tall problem: A's column c enters times cscale[c], a
// power of two that puts the column's largest entry in [1, 2), so FP16's
// range holds it; the caller divides the sketch's column c by the same power.
template <typename TA, int KB, int ST>
__global__ void __launch_bounds__(256, ST == 256 ? 2 : 1) k_sketch_gemm_f16(const _Float16* __restrict__ X,
                                                         int64_t s, int64_t kc, int64_t ldx,
                                                         int64_t ksz,
                                                         const TA* __restrict__ A, int64_t lda,
                                                         int64_t r0, int64_t ncol, int sR, int cR,
                                                         int pc, float* __restrict__ Y, int first,
                                                         const float* __restrict__ cscale) {
  sketch_gemm_body<_Float16, TA, false, KB, ST>(reinterpret_cast<const uint16_t*>(X), s, kc, ldx, ksz, A, lda,
                                                r0, ncol, sR, cR, pc, Y, first, cscale);
}

// Y (count floats) = [Y +] sum_z part[z] in order z = 0, 1, ... (deterministic).
__global__ void k_sketch_reduce(const float* __restrict__ part, int nz, int64_t count,
                                float* __restrict__ Y, int first) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = first ? 0.f : Y[i];
  for (int z = 0; z < nz; ++z) acc += part[int64_t(z) * count + i];
  Y[i] = acc;
}

__global__ void k_f32_to_f64(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = double(src[i]);
}

// dst (s x ncol) = src / cscale[column]: undoes the power-of-two column scaling
// of the FP16 product exactly.
__global__ void k_f32_to_f64_cols(const float* __restrict__ src, double* __restrict__ dst, int64_t s,
                                  int64_t ncol, const float* __restrict__ cscale) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < s * ncol) dst[i] = double(src[i]) / double(cscale[i / s]);
}

// cscale[c] = 2^-e with e the exponent of column c's largest |A(r, c)|
// (largest entry scaled into [1, 2)); 1 for a zero or non-finite column.  One
// block per column.
template <typename TA>
__global__ void __launch_bounds__(256) k_col_pow2(const TA* __restrict__ A, int64_t m, int64_t lda,
                                                  float* __restrict__ cscale) {
  __shared__ float red[4];
  const int64_t c = blockIdx.x;
  float mx = 0.f;
  for (int64_t r = threadIdx.x; r < m; r += 256) mx = fmaxf(mx, fabsf(float(A[r + c * lda])));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float v = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    cscale[c] = (v > 0.f && v < INFINITY) ? ldexpf(1.f, -ilogbf(v)) : 1.f;
  }
}

// ---------------------------------------------------------------- launchers --
int launch_srht_rows(uint64_t seed, int k, int64_t s, int32_t* rows, int32_t* bstart, int bbits,
                     hipStream_t st) {
  if (k < 0 || k > ROWS_KMAX || bbits < 0 || bbits > k || s < 0 || s > (int64_t(1) << k)) {
    set_error("internal: SRHT row sampler needs 0 <= bbits <= k <= 18 and s <= 2^k");
    return TIK_EINVAL;
  }
  // signs live right after the bucket table (caller sized it)
  uint32_t* signs = reinterpret_cast<uint32_t*>(bstart + (1 << (k - bbits)) + 1);
  ProfScope ps("sketch", st);
  hipLaunchKernelGGL(k_srht_rows, dim3(1), dim3(1024), 0, st, seed, k, s, rows, bstart, bbits,
                     signs);
  TIK_LAUNCHED("k_srht_rows");
  return TIK_OK;
}

static const uint32_t* signs_of(const int32_t* bstart, int k, int bbits) {
  return reinterpret_cast<const uint32_t*>(bstart + (1 << (k - bbits)) + 1);
}

int launch_srht_single(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int k,
                       uint64_t seed, const int32_t* rows, int64_t s, double* Y, hipStream_t st) {
  (void)seed;
  const int32_t* bstart = rows + s;  // layout set by the caller: rows | bstart | signs
  const uint32_t* signs = signs_of(bstart, k, k);
  const double scale = 1.0 / sqrt(double(s));
  const size_t lds = sizeof(double) << k;
  ProfScope ps("sketch", st);
  if (a_f32)
    hipLaunchKernelGGL(k_srht_single<float>, dim3(unsigned(n)), dim3(256), lds, st,
                       static_cast<const float*>(A), m, lda, k, signs, rows, s, scale, Y);
  else
    hipLaunchKernelGGL(k_srht_single<double>, dim3(unsigned(n)), dim3(256), lds, st,
                       static_cast<const double*>(A), m, lda, k, signs, rows, s, scale, Y);
  TIK_LAUNCHED("k_srht_single");
  return TIK_OK;
}

template <typename TA>
static int pass1_dispatch(const TA* A, int64_t m, int64_t lda, int64_t c0, int64_t nc, int abits,
                          int bbits, const uint32_t* signs, double* T, hipStream_t st) {
  dim3 grid(unsigned(cdiv(int64_t(1) << bbits, 256)), unsigned(nc));
  switch (abits) {
    case 1: hipLaunchKernelGGL((k_srht_pass1<TA, 1>), grid, dim3(256), 0, st, A, m, lda, c0, bbits, signs, T); break;
    case 2: hipLaunchKernelGGL((k_srht_pass1<TA, 2>), grid, dim3(256), 0, st, A, m, lda, c0, bbits, signs, T); break;
    case 3: hipLaunchKernelGGL((k_srht_pass1<TA, 3>), grid, dim3(256), 0, st, A, m, lda, c0, bbits, signs, T); break;
    case 4: hipLaunchKernelGGL((k_srht_pass1<TA, 4>), grid, dim3(256), 0, st, A, m, lda, c0, bbits, signs, T); break;
    case 5: hipLaunchKernelGGL((k_srht_pass1<TA, 5>), grid, dim3(256), 0, st, A, m, lda, c0, bbits, signs, T); break;
    default: set_error("SRHT: unsupported split"); return TIK_ENOTSUP;
  }
  TIK_LAUNCHED("k_srht_pass1");
  return TIK_OK;
}

// Column chunk [c0, c0 + nc) of the two-pass transform.  rows | bstart | signs
// are laid out consecutively by the caller.
int launch_srht_twopass(const void* A, int a_f32, int64_t m, int64_t lda, int64_t c0, int64_t nc,
                        int k, int bbits, const int32_t* rows, int64_t s, double* T, double* Y,
                        hipStream_t st) {
  const int32_t* bstart = rows + s;
  const uint32_t* signs = signs_of(bstart, k, bbits);
  const int abits = k - bbits;
  ProfScope ps("sketch", st);
  if (a_f32)
    TIK_TRY(pass1_dispatch(static_cast<const float*>(A), m, lda, c0, nc, abits, bbits, signs, T, st));
  else
    TIK_TRY(pass1_dispatch(static_cast<const double*>(A), m, lda, c0, nc, abits, bbits, signs, T, st));
  const size_t lds = sizeof(double) << bbits;
  hipLaunchKernelGGL(k_srht_pass2, dim3(1u << abits, unsigned(nc)), dim3(256), lds, st, T, c0, k,
                     bbits, rows, bstart, s, 1.0 / sqrt(double(s)), Y);
  TIK_LAUNCHED("k_srht_pass2");
  return TIK_OK;
}

bool srht_cols_ok(int k, int64_t n, int64_t s) {
  return k >= SRC_BITS && k <= 30 && n >= kSrhtColsMinN && s <= 8192;
}

template <typename TA>
static void srht_cols_launch(const TA* A, int64_t m, int64_t n, int64_t lda, const uint32_t* signs,
                             const int32_t* rows, int64_t s, double scale, double* Y,
                             hipStream_t st) {
  const dim3 grid = dim3(unsigned(n)), block = dim3(SRC_T);
  static_assert(8192 == 16 * SRC_T, "sampled rows per thread");
  if (s <= 8 * SRC_T)
    hipLaunchKernelGGL((k_srht_cols<TA, 8>), grid, block, 0, st, A, m, lda, signs, rows, s, scale, Y);
  else
    hipLaunchKernelGGL((k_srht_cols<TA, 16>), grid, block, 0, st, A, m, lda, signs, rows, s, scale, Y);
}

// Column-resident transform of every column; rows | bstart | signs laid out by
// the caller with buckets of 2^bbits rows.
int launch_srht_cols(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int k, int bbits,
                     const int32_t* rows, int64_t s, double* Y, hipStream_t st) {
  if (!srht_cols_ok(k, n, s)) {
    set_error("internal: column-resident SRHT outside its range");
    return TIK_EINVAL;
  }
  const int32_t* bstart = rows + s;
  const uint32_t* signs = signs_of(bstart, k, bbits);
  const double scale = 1.0 / sqrt(double(s));
  ProfScope ps("sketch", st);
  if (a_f32)
    srht_cols_launch(static_cast<const float*>(A), m, n, lda, signs, rows, s, scale, Y, st);
  else
    srht_cols_launch(static_cast<const double*>(A), m, n, lda, signs, rows, s, scale, Y, st);
  TIK_LAUNCHED("k_srht_cols");
  return TIK_OK;
}

int launch_gauss_gen(uint64_t seed, int64_t s, int64_t r0, int64_t kc, int64_t ldx, void* Xc,
                     int kind, hipStream_t st) {
  if (ldx < kc || (kind == 0 && ldx != kc)) {
    set_error("internal: Gaussian chunk pitch");
    return TIK_EINVAL;
  }
  const int64_t total = ((s + 3) >> 2) * kc;
  const double scale = 1.0 / sqrt(double(s));
  ProfScope ps("sketch", st);
  if (kind == 1)
    hipLaunchKernelGGL(k_gauss_gen_bf16, dim3(unsigned(cdiv(total, 256))), dim3(256), 0, st, seed,
                       s, r0, kc, ldx, float(scale), static_cast<__hip_bfloat16*>(Xc));
  else if (kind == 2)
    hipLaunchKernelGGL(k_gauss_gen_f16, dim3(unsigned(cdiv(total, 256))), dim3(256), 0, st, seed,
                       s, r0, kc, ldx, float(scale), static_cast<_Float16*>(Xc));
  else
    hipLaunchKernelGGL(k_gauss_gen<double>, dim3(unsigned(cdiv(total, 256))), dim3(256), 0, st,
                       seed, s, r0, kc, scale, static_cast<double*>(Xc));
  TIK_LAUNCHED("k_gauss_gen");
  return TIK_OK;
}

int launch_sketch_gemm_f64(const double* Xc, int64_t s, int64_t kc, const void* A, int a_f32,
                           int64_t lda, int64_t r0, int64_t ncol, int wide, double* Y,
                           hipStream_t st) {
  dim3 grid(unsigned(cdiv(s, 64)), unsigned(cdiv(ncol, 64)));
  ProfScope ps("sketch", st);
  if (a_f32) {
    if (wide) hipLaunchKernelGGL((k_sketch_gemm64<float, true>), grid, dim3(256), 0, st, Xc, s, kc, static_cast<const float*>(A), lda, r0, ncol, Y);
    else      hipLaunchKernelGGL((k_sketch_gemm64<float, false>), grid, dim3(256), 0, st, Xc, s, kc, static_cast<const float*>(A), lda, r0, ncol, Y);
  } else {
    if (wide) hipLaunchKernelGGL((k_sketch_gemm64<double, true>), grid, dim3(256), 0, st, Xc, s, kc, static_cast<const double*>(A), lda, r0, ncol, Y);
    else      hipLaunchKernelGGL((k_sketch_gemm64<double, false>), grid, dim3(256), 0, st, Xc, s, kc, static_cast<const double*>(A), lda, r0, ncol, Y);
  }
  TIK_LAUNCHED("k_sketch_gemm64");
  return TIK_OK;
}

// Sketch rows per output tile: 256 (it halves the A loads per flop, at two
// blocks per CU instead of three) once the sketch has 4096 rows or more, where
// it measured faster (s = 8000: 27.9 -> 24.8 ms); 128 below (s from 400 to
// 4000 in a ragged batch: 120 ms either way with this threshold, 138 ms with
// 256-row tiles from s = 1024 on).
constexpr int SK_KB = 32;    // k per step of the BF16 sketch product
constexpr int64_t SK_ST256_MIN = 4096;
static int sketch_bf16_st(int64_t s) { return s >= SK_ST256_MIN ? 256 : 128; }

// K splits of one BF16 sketch launch: enough blocks to fill the chip when the
// output has few tiles, at least 512 k per split, partial slices within
// `part_cap` floats.
int sketch_bf16_splits(int64_t s, int64_t ncol, int64_t kc, int64_t part_cap) {
  const int64_t tiles = cdiv(s, sketch_bf16_st(s)) * cdiv(ncol, 128);
  int64_t z = std::max<int64_t>(1, std::min<int64_t>(1024 / std::max<int64_t>(1, tiles), kc / 512));
  if (z > 1) z = std::min<int64_t>(z, part_cap / std::max<int64_t>(1, s * ncol));
  return int(std::max<int64_t>(1, z));
}

int launch_sketch_gemm_bf16(const void* Xc, int64_t s, int64_t kc, int64_t ldx, const void* A,
                            int a_f32, int64_t lda, int64_t r0, int64_t ncol, int wide, float* Yacc,
                            int first, float* part, int64_t part_cap, hipStream_t st,
                            const float* cscale) {
  if (cscale && wide) {
    set_error("internal: the FP16 sketch product is for tall problems");
    return TIK_EINVAL;
  }
  int nz = sketch_bf16_splits(s, ncol, kc, part_cap);
  const int64_t ksz = cdiv(cdiv(kc, nz), SK_KB) * SK_KB;
  nz = int(cdiv(kc, ksz));
  float* dst = nz > 1 ? part : Yacc;
  // XCD split ps x pc of the S x C tile grid: X panels are fetched by pc XCDs,
  // A panels by ps; take the split with the fewest bytes
  const int ST = sketch_bf16_st(s);
  const int64_t S = cdiv(s, ST), C = cdiv(ncol, 128);
  const double xb = double(s) * double(ksz) * 2.0;
  const double ab = double(ncol) * double(ksz) * (a_f32 ? 4.0 : 8.0);
  int pc = 1;
  double best = -1.0;
  for (int c = 1; c <= 8; c *= 2) {
    const int ps = 8 / c;
    if ((c > 1 && C < c) || (ps > 1 && S < ps)) continue;
    const double cost = xb * c + ab * ps;
    if (best < 0.0 || cost < best) {
      best = cost;
      pc = c;
    }
  }
  const int sR = int(cdiv(S, 8 / pc)), cR = int(cdiv(C, pc));
  const dim3 grid = dim3(unsigned(8 * sR * cR), 1u, unsigned(nz));
  const __hip_bfloat16* X = static_cast<const __hip_bfloat16*>(Xc);
  ProfScope ps("sketch", st);
#define TIK_SKG(TAV, WV, STV)                                                                   \
  hipLaunchKernelGGL((k_sketch_gemm_bf16<TAV, WV, SK_KB, STV>), grid, dim3(256), 0, st, X, s, kc, \
                     ldx, ksz, static_cast<const TAV*>(A), lda, r0, ncol, sR, cR, pc, dst, first)
#define TIK_SKH(TAV, STV)                                                                       \
  hipLaunchKernelGGL((k_sketch_gemm_f16<TAV, SK_KB, STV>), grid, dim3(256), 0, st,              \
                     static_cast<const _Float16*>(Xc), s, kc, ldx, ksz, static_cast<const TAV*>(A), lda, r0, \
                     ncol, sR, cR, pc, dst, first, cscale)
  if (cscale) {
    if (ST == 256) { if (a_f32) TIK_SKH(float, 256); else TIK_SKH(double, 256); }
    else           { if (a_f32) TIK_SKH(float, 128); else TIK_SKH(double, 128); }
  } else if (ST == 256) {
    if (a_f32) { if (wide) TIK_SKG(float, true, 256); else TIK_SKG(float, false, 256); }
    else       { if (wide) TIK_SKG(double, true, 256); else TIK_SKG(double, false, 256); }
  } else {
    if (a_f32) { if (wide) TIK_SKG(float, true, 128); else TIK_SKG(float, false, 128); }
    else       { if (wide) TIK_SKG(double, true, 128); else TIK_SKG(double, false, 128); }
  }
#undef TIK_SKG
#undef TIK_SKH
  TIK_LAUNCHED("k_sketch_gemm_16");
  if (nz > 1) {
    const int64_t count = s * ncol;
    hipLaunchKernelGGL(k_sketch_reduce, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, st, part,
                       nz, count, Yacc, first);
    TIK_LAUNCHED("k_sketch_reduce");
  }
  return TIK_OK;
}

// ------------------------------------------------------ sparse embedding ---
// X (s x m) with zeta nonzeros per column, each +-1/sqrt(zeta): column i (row i
// of A) puts nonzero t < zeta in a uniformly drawn row of the t-th of zeta
// consecutive row blocks of X (block sizes differ by at most one), so the
// zeta rows are distinct and every column of X has unit norm, E[X^T X] = I.
// map[i zeta + t] = row | (sign bit 31).
__global__ void __launch_bounds__(256) k_sparse_map(uint64_t seed, int64_t m, int64_t s, int zeta,
                                                    int32_t* __restrict__ map) {
  const uint2 key = seed_key(seed);
  const int64_t bs = s / zeta, rem = s % zeta;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < m * zeta; e += int64_t(gridDim.x) * 256) {
    const int64_t i = e / zeta;
    const int t = int(e % zeta);
    const uint4 r = philox4x32_10(make_uint4(uint32_t(i), uint32_t(i >> 32) ^ (uint32_t(t) << 16), TAG_SPAR, 0u),
                                  key);
    const int64_t len = bs + (t < rem ? 1 : 0);
    const int64_t start = int64_t(t) * bs + min<int64_t>(t, rem);
    const int64_t row = start + int64_t((uint64_t(r.x) * uint64_t(len)) >> 32);
    map[e] = int32_t(row) | int32_t((r.y & 1u) << 31);
  }
}

// Y[:, c] = X A[:, c] for one column c per block: the column streams through
// once (coalesced) and its entries are added into the s rows of Y kept in LDS.
// The additions into one row arrive in no fixed order, so Y is X A up to the
// rounding order of FP64 sums (X itself is fixed by the seed).
// Rows of Y per block: larger sketches split Y's rows over several blocks per
// column, each reading the column (the blocks of one column are adjacent).
static constexpr int64_t SP_ROWS = 8192;

template <typename TA>
__global__ void __launch_bounds__(512) k_sparse_apply(const TA* __restrict__ A, int64_t m, int64_t lda,
                                                      int64_t s, int zeta, int nr,
                                                      const int32_t* __restrict__ map,
                                                      double* __restrict__ Y) {
  __shared__ double acc[SP_ROWS];
  const int64_t c = blockIdx.x / nr;
  const int64_t r0 = int64_t(blockIdx.x % nr) * SP_ROWS;
  const int64_t rn = min<int64_t>(SP_ROWS, s - r0);
  for (int64_t r = threadIdx.x; r < rn; r += 512) acc[r] = 0.0;
  __syncthreads();
  const TA* __restrict__ col = A + c * lda;
  for (int64_t i = threadIdx.x; i < m; i += 512) {
    const double a = double(col[i]);
    for (int t = 0; t < zeta; ++t) {
      const int32_t e = map[i * zeta + t];
      const int64_t r = int64_t(e & 0x7fffffff) - r0;
      if (r >= 0 && r < rn) atomicAdd(&acc[r], e < 0 ? -a : a);
    }
  }
  __syncthreads();
  const double sc = 1.0 / sqrt(double(zeta));
  for (int64_t r = threadIdx.x; r < rn; r += 512) Y[r0 + r + c * s] = acc[r] * sc;
}

int launch_sparse_sketch(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, int64_t s,
                         int zeta, uint64_t seed, int32_t* map, double* Y, hipStream_t st) {
  ProfScope ps("sketch", st);
  const int64_t tot = m * zeta;
  hipLaunchKernelGGL(k_sparse_map, dim3(unsigned(std::min<int64_t>(cdiv(tot, 256), 65536))), dim3(256), 0, st,
                     seed, m, s, zeta, map);
  TIK_LAUNCHED("k_sparse_map");
  const int nr = int(cdiv(s, SP_ROWS));
  const dim3 g(unsigned(n * nr));
  if (a_f32)
    hipLaunchKernelGGL(k_sparse_apply<float>, g, dim3(512), 0, st, static_cast<const float*>(A), m, lda, s,
                       zeta, nr, map, Y);
  else
    hipLaunchKernelGGL(k_sparse_apply<double>, g, dim3(512), 0, st, static_cast<const double*>(A), m, lda,
                       s, zeta, nr, map, Y);
  TIK_LAUNCHED("k_sparse_apply");
  return TIK_OK;
}

int launch_col_pow2(const void* A, int a_f32, int64_t m, int64_t n, int64_t lda, float* cscale,
                    hipStream_t st) {
  ProfScope ps("sketch", st);
  if (a_f32)
    hipLaunchKernelGGL(k_col_pow2<float>, dim3(unsigned(n)), dim3(256), 0, st, static_cast<const float*>(A), m,
                       lda, cscale);
  else
    hipLaunchKernelGGL(k_col_pow2<double>, dim3(unsigned(n)), dim3(256), 0, st, static_cast<const double*>(A),
                       m, lda, cscale);
  TIK_LAUNCHED("k_col_pow2");
  return TIK_OK;
}

int launch_f32_to_f64_cols(const float* src, double* dst, int64_t s, int64_t ncol, const float* cscale,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_f64_cols, dim3(unsigned(cdiv(s * ncol, 256))), dim3(256), 0, st, src, dst, s,
                     ncol, cscale);
  TIK_LAUNCHED("k_f32_to_f64");
  return TIK_OK;
}

int launch_f32_to_f64(const float* src, double* dst, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(unsigned(cdiv(count, 256))), dim3(256), 0, st, src, dst,
                     count);
  TIK_LAUNCHED("k_f32_to_f64");
  return TIK_OK;
}

}  // namespace tik
