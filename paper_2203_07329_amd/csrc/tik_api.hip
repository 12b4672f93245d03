// C ABI entry points of libtik: argument validation, workspace planning and
// stream-ordered orchestration of the sketch, preconditioner and solve kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "tik_internal.h"

#include <atomic>

namespace tik {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static thread_local std::vector<double> g_times;    // ms, NaN where not recorded
static thread_local int64_t g_t0 = -1;               // tstart of the call's first group
static std::atomic<int> g_opt_times{0};
bool option_record_times() { return g_opt_times.load(std::memory_order_relaxed) != 0; }
void times_reset(int64_t count) {
  g_times.assign(size_t(std::max<int64_t>(count, 0)), std::nan(""));
  g_t0 = -1;
}
void times_note(const Scal* hs, int J, int N, const std::vector<int>& pidx, const std::vector<int>& lsel,
                int Ntot, hipStream_t st) {
  int dev = 0;
  int khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return;
  (void)st;
  if (g_t0 < 0 && J > 0) g_t0 = hs[0].tstart;
  for (int j = 0; j < J; ++j) {
    const size_t g = size_t(pidx[size_t(j / N)]) * size_t(Ntot) + size_t(lsel[size_t(j % N)]);
    if (g < g_times.size()) g_times[g] = double(hs[j].tdone - g_t0) / double(khz);
  }
}

static thread_local int32_t g_split32 = 0, g_split64 = 0;
void note_split(int32_t fp32, int32_t fp64) {
  g_split32 += fp32;
  g_split64 += fp64;
}
void last_split(int32_t* fp32, int32_t* fp64) {
  *fp32 = g_split32;
  *fp64 = g_split64;
}

static int fail(int rc, const std::string& msg) {
  g_err = msg;
  return rc;
}

// ------------------------------------------------------------- profiling ---
namespace {
struct ProfFamily {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double done_ms = 0.0;
  int64_t done_n = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfFamily> g_prof;
std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> g_open;
}  // namespace

ProfScope::ProfScope(const char* family, hipStream_t s) : slot(-1), st(s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(a, st);
  g_open.push_back({family, {a, b}});
  slot = int(g_open.size()) - 1;
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto& o = g_open[size_t(slot)];
  (void)hipEventRecord(o.second.second, st);
  g_prof[o.first].ev.push_back(o.second);
  o.second = {nullptr, nullptr};
}

bool prof_active() { return g_prof_on; }

// ---------------------------------------------------------------- options --
namespace {
std::atomic<int> g_opt_chunk{4};
std::atomic<int64_t> g_opt_pivot{0};
std::atomic<int> g_opt_nnz{1};
std::atomic<int> g_opt_cqr{1};
std::atomic<int> g_opt_srht_cols{1};
std::atomic<int> g_opt_gn_tail{1};
}
int option_sparse_nnz() { return g_opt_nnz.load(std::memory_order_relaxed); }
int option_cholqr_panels() { return g_opt_cqr.load(std::memory_order_relaxed); }
int option_srht_cols() { return g_opt_srht_cols.load(std::memory_order_relaxed); }
int option_gemm_n_tail() { return g_opt_gn_tail.load(std::memory_order_relaxed); }
int option_chunk() { return g_opt_chunk.load(std::memory_order_relaxed); }
int64_t option_pivot_ulps() { return g_opt_pivot.load(std::memory_order_relaxed); }

void prof_drop_last(const char* family) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto it = g_prof.find(family);
  if (it == g_prof.end() || it->second.ev.empty()) return;
  const auto e = it->second.ev.back();
  it->second.ev.pop_back();
  (void)hipEventDestroy(e.first);
  (void)hipEventDestroy(e.second);
}

// ---------------------------------------------------------------- helpers --
static bool tall(const tik_problem& p) { return p.m >= p.n; }

static int validate_problems(const tik_problem* p, int32_t nprob, const char* fn) {
  if (!p || nprob < 1) return fail(TIK_EINVAL, std::string(fn) + ": need at least one problem");
  for (int32_t k = 0; k < nprob; ++k) {
    const tik_problem& q = p[k];
    const std::string at = std::string(fn) + ": problem " + std::to_string(k) + ": ";
    if (q.m < 1 || q.n < 1) return fail(TIK_EINVAL, at + "m and n must be >= 1");
    if (q.lda < q.m) return fail(TIK_EINVAL, at + "lda must be >= m");
    if (q.a_dtype != TIK_F64 && q.a_dtype != TIK_F32)
      return fail(TIK_EINVAL, at + "a_dtype must be TIK_F64 or TIK_F32");
    if (q.reserved != 0) return fail(TIK_EINVAL, at + "reserved must be 0");
    if (!q.A || !q.b) return fail(TIK_EINVAL, at + "A and b must be device pointers");
    if (q.m > (int64_t(1) << 31) || q.n > (int64_t(1) << 31))
      return fail(TIK_EINVAL, at + "dimensions above 2^31 are not supported");
    if (tall(q) != tall(p[0]))
      return fail(TIK_EINVAL, std::string(fn) + ": all problems must be tall (m >= n) or all wide");
    if (q.a_dtype != p[0].a_dtype)
      return fail(TIK_EINVAL, std::string(fn) + ": all problems must share one storage type");
  }
  return TIK_OK;
}

static int check_ws(void* dws, size_t dws_bytes, size_t need, const char* fn) {
  if (need > 0 && !dws) return fail(TIK_EWORKSPACE, std::string(fn) + ": workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dws) % 256 != 0)
    return fail(TIK_EWORKSPACE, std::string(fn) + ": workspace must be 256-byte aligned");
  if (dws_bytes < need)
    return fail(TIK_EWORKSPACE, std::string(fn) + ": workspace of " + std::to_string(dws_bytes) +
                                    " bytes, need " + std::to_string(need));
  return TIK_OK;
}

static int ilog2_ceil(int64_t v) {
  int k = 0;
  while ((int64_t(1) << k) < v) ++k;
  return k;
}

static constexpr int SRHT_MAX_K = 18;
static constexpr int64_t SRHT_MAX_S = 16384;
static constexpr size_t SCRATCH_CHUNK = size_t(256) << 20;
static constexpr int64_t kBf16PartCap = int64_t(32) << 20;   // floats of split-K partials

// ------------------------------------------------------------------ lanes --
// The per-problem work of a batch (sketch, Gram, factorization) is a chain of
// small launches per problem.  Problems are spread over up to kLanes streams
// the library owns (default priority, created once per device), each with its
// own scratch: forked from the caller's stream with an event, joined back with
// one event per lane, so the caller sees ordinary stream order.
static constexpr int kLanes = 4;

namespace {
std::mutex g_lane_mu;
std::map<int, std::vector<hipStream_t>> g_lane_streams;

struct Lanes {
  hipStream_t main = nullptr;
  int n = 1;
  hipStream_t s[kLanes] = {};
  hipEvent_t ev[kLanes + 1] = {};
  bool forked = false;

  int fork(hipStream_t st, int want) {
    main = st;
    n = std::max(1, std::min(kLanes, want));
    s[0] = st;
    if (n == 1) return TIK_OK;
    int dev = 0;
    TIK_HIP(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> lk(g_lane_mu);
      auto& pool = g_lane_streams[dev];
      while (int(pool.size()) < kLanes) {
        hipStream_t x;
        TIK_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        pool.push_back(x);
      }
      for (int i = 0; i < n; ++i) s[i] = pool[size_t(i)];
    }
    for (int i = 0; i <= n; ++i) TIK_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    forked = true;
    TIK_HIP(hipEventRecord(ev[n], st));
    for (int i = 0; i < n; ++i) TIK_HIP(hipStreamWaitEvent(s[i], ev[n], 0));
    return TIK_OK;
  }
  hipStream_t at(int k) const { return s[k % n]; }
  int join() {
    if (!forked) return TIK_OK;
    forked = false;
    for (int i = 0; i < n; ++i) {
      TIK_HIP(hipEventRecord(ev[i], s[i]));
      TIK_HIP(hipStreamWaitEvent(main, ev[i], 0));
    }
    for (int i = 0; i <= n; ++i) (void)hipEventDestroy(ev[i]);
    return TIK_OK;
  }
  ~Lanes() {
    if (forked) (void)join();
  }
};
}  // namespace

// --------------------------------------------------------------- sketch ----
struct SketchPlan {
  std::vector<double*> Y;
  std::vector<int64_t> yrows, ycols;
  // scratch, one set per lane
  int32_t* rows[kLanes] = {};   // SRHT: rows | bucket starts | sign words
  double* T[kLanes] = {};       // SRHT two-pass scratch
  double* Xc[kLanes] = {};      // Gaussian X chunk (FP64 or BF16)
  float* Yacc[kLanes] = {};     // BF16 sketches: FP32 accumulator
  float* Ypart[kLanes] = {};    // BF16 sketches: split-K partial products
  float* cscale[kLanes] = {};   // FP16 sketches: power-of-two column scales of A
  int64_t part_cap = 0;         // floats in each Ypart
  int lanes = 1;
  int64_t tcols = 0, kc = 0;
};

// long-dimension rows of the Gaussian X generated per chunk for problem q
static int64_t gauss_chunk(const tik_problem& q, int64_t s, int32_t sdt) {
  const int64_t longdim = tall(q) ? q.m : q.n;
  const bool h16 = sdt == TIK_BF16 || sdt == TIK_F16;
  const size_t esz = h16 ? 2 : sizeof(double);
  int64_t kc = int64_t(SCRATCH_CHUNK / (esz * size_t(s)));
  kc = std::max<int64_t>(64, std::min<int64_t>(longdim, kc));
  if (h16 && kc < longdim) kc = std::max<int64_t>(32, kc / 32 * 32);
  return kc;
}

// row pitch of a Gaussian X chunk: 16-bit rows start 16-byte aligned so the
// sketch product fetches them with vector loads
static int64_t gauss_pitch(int64_t kc, int32_t sdt) {
  return (sdt == TIK_BF16 || sdt == TIK_F16) ? cdiv(kc, 8) * 8 : kc;
}

// the column-resident transform where it applies and is not switched off
static bool srht_cols_use(int k, int64_t n, int64_t s) {
  return option_srht_cols() && srht_cols_ok(k, n, s);
}

static int sketch_plan(const tik_problem* p, int32_t nprob, int32_t embed, int32_t sdt,
                       const int64_t* s, Arena& a, SketchPlan& sp) {
  sp.Y.assign(size_t(nprob), nullptr);
  sp.yrows.assign(size_t(nprob), 0);
  sp.ycols.assign(size_t(nprob), 0);
  int64_t rows_ints = 0, tsz = 0, xsz = 0, ysz = 0, csz = 0;
  for (int32_t k = 0; k < nprob; ++k) {
    const bool t = tall(p[k]);
    sp.yrows[k] = s[k];
    sp.ycols[k] = t ? p[k].n : p[k].m;
    sp.Y[k] = a.take<double>(size_t(s[k]) * size_t(sp.ycols[k]));
    if (embed == TIK_SPARSE) {
      rows_ints = std::max<int64_t>(rows_ints, p[k].m * int64_t(option_sparse_nnz()));
    } else if (embed == TIK_SRHT) {
      const int kk = ilog2_ceil(p[k].m);
      const int bb = kk <= 13 ? kk : 13;
      rows_ints = std::max<int64_t>(rows_ints, s[k] + (int64_t(1) << (kk - bb)) + 1 +
                                                   (((int64_t(1) << kk) + 31) >> 5));
      if (kk > 13 && !srht_cols_use(kk, p[k].n, s[k])) {
        const int64_t cols = std::max<int64_t>(
            1, std::min<int64_t>(p[k].n, int64_t(SCRATCH_CHUNK / (sizeof(double) << kk))));
        sp.tcols = std::max(sp.tcols, cols);
        tsz = std::max<int64_t>(tsz, cols << kk);
      }
    } else {
      const bool h16 = sdt == TIK_BF16 || sdt == TIK_F16;
      const size_t esz = h16 ? 2 : sizeof(double);
      xsz = std::max<int64_t>(xsz, int64_t(cdiv(gauss_pitch(gauss_chunk(p[k], s[k], sdt), sdt) *
                                                s[k] * int64_t(esz), 8)));
      if (sdt == TIK_F16) csz = std::max<int64_t>(csz, sp.ycols[k]);
      if (h16) {
        ysz = std::max<int64_t>(ysz, s[k] * sp.ycols[k]);
        const int64_t kc = gauss_chunk(p[k], s[k], sdt);
        const int z = sketch_bf16_splits(s[k], sp.ycols[k], kc, kBf16PartCap);
        if (z > 1) sp.part_cap = std::max<int64_t>(sp.part_cap, int64_t(z) * s[k] * sp.ycols[k]);
      }
    }
  }
  sp.lanes = std::max(1, std::min<int>(kLanes, nprob));
  for (int l = 0; l < sp.lanes; ++l) {
    if (rows_ints) sp.rows[l] = a.take<int32_t>(size_t(rows_ints));
    if (tsz) sp.T[l] = a.take<double>(size_t(tsz));
    if (xsz) sp.Xc[l] = a.take<double>(size_t(xsz));
    if (ysz) sp.Yacc[l] = a.take<float>(size_t(ysz));
    if (sp.part_cap) sp.Ypart[l] = a.take<float>(size_t(sp.part_cap));
    if (csz) sp.cscale[l] = a.take<float>(size_t(csz));
  }
  return TIK_OK;
}

static int sketch_validate(const tik_problem* p, int32_t nprob, int32_t embed, int32_t sdt,
                           const int64_t* s) {
  TIK_TRY(validate_problems(p, nprob, "tik_sketch"));
  if (embed != TIK_SRHT && embed != TIK_GAUSS && embed != TIK_SPARSE)
    return fail(TIK_EINVAL, "tik_sketch: embed must be TIK_SRHT, TIK_GAUSS or TIK_SPARSE");
  if (sdt != TIK_F64 && sdt != TIK_BF16 && sdt != TIK_F16)
    return fail(TIK_EINVAL, "tik_sketch: sketch_dtype must be TIK_F64, TIK_BF16 or TIK_F16");
  if ((sdt == TIK_BF16 || sdt == TIK_F16) && embed != TIK_GAUSS)
    return fail(TIK_EINVAL, "tik_sketch: 16-bit sketches need the Gaussian embedding");
  if (sdt == TIK_F16)
    for (int32_t k = 0; k < nprob; ++k)
      if (!tall(p[k]))
        return fail(TIK_ENOTSUP, "tik_sketch: the FP16 sketch is implemented for tall problems only");
  if (!s) return fail(TIK_EINVAL, "tik_sketch: s is NULL");
  for (int32_t k = 0; k < nprob; ++k) {
    const int64_t longdim = tall(p[k]) ? p[k].m : p[k].n;
    if (s[k] < 1 || s[k] > longdim)
      return fail(TIK_EINVAL, "tik_sketch: problem " + std::to_string(k) +
                                  ": sketch size must lie in [1, long dimension]");
    if (embed == TIK_SRHT) {
      if (!tall(p[k]))
        return fail(TIK_ENOTSUP, "tik_sketch: the SRHT is implemented for tall problems only");
      if (ilog2_ceil(p[k].m) > SRHT_MAX_K)
        return fail(TIK_ENOTSUP, "tik_sketch: SRHT needs m <= 2^18");
      if (s[k] > SRHT_MAX_S) return fail(TIK_ENOTSUP, "tik_sketch: SRHT needs s <= 16384");
    }
    if (embed == TIK_SPARSE) {
      if (!tall(p[k]))
        return fail(TIK_ENOTSUP, "tik_sketch: the sparse embedding is implemented for tall problems only");
      if (s[k] < option_sparse_nnz())
        return fail(TIK_EINVAL, "tik_sketch: the sparse embedding needs s >= its nonzeros per column");
      if (p[k].m * int64_t(option_sparse_nnz()) >= (int64_t(1) << 31))
        return fail(TIK_ENOTSUP, "tik_sketch: the sparse embedding needs m * nonzeros < 2^31");
    }
  }
  return TIK_OK;
}

// ----------------------------------------------------- no-allocation solve --
// Workspace of tik_lsqr_batch_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel or copy: it uses the device address hipGetSymbolAddress returns,
// looked up once per device with that device current, on the entry point's
// first call there.
static constexpr size_t kStaticBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device: the address of `scratch` there
thread_local bool t_noalloc = false;
struct NoAllocScope {
  NoAllocScope() { t_noalloc = true; }
  ~NoAllocScope() { t_noalloc = false; }
};
}  // namespace

bool noalloc_active() { return t_noalloc; }

static int scratch_address(void** out) {
  int dev = 0;
  TIK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[size_t(dev)]) {
    void* ptr = nullptr;
    TIK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(TIK_EHIP, "hipGetSymbolAddress returned a null address for the static workspace");
    g_scratch_ptr[size_t(dev)] = ptr;
  }
  *out = g_scratch_ptr[size_t(dev)];
  return TIK_OK;
}

}  // namespace tik

using namespace tik;

extern "C" {

const char* tik_last_error(void) { return g_err.c_str(); }

int tik_version(void) { return 200; }

int tik_set_option(const char* name, int64_t value) {
  if (!name) return fail(TIK_EINVAL, "tik_set_option: name is NULL");
  if (std::string(name) == "graph_chunk") {
    if (value < 0 || value > 64) return fail(TIK_EINVAL, "tik_set_option: graph_chunk must be 0..64");
    g_opt_chunk.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "sparse_nnz") {
    if (value < 1 || value > 16) return fail(TIK_EINVAL, "tik_set_option: sparse_nnz must be 1..16");
    g_opt_nnz.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "record_times") {
    if (value < 0 || value > 1) return fail(TIK_EINVAL, "tik_set_option: record_times must be 0 or 1");
    g_opt_times.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "cholqr_panels") {
    if (value < 0 || value > 1) return fail(TIK_EINVAL, "tik_set_option: cholqr_panels must be 0 or 1");
    g_opt_cqr.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "gemm_n_tail") {
    if (value < 0 || value > 1) return fail(TIK_EINVAL, "tik_set_option: gemm_n_tail must be 0 or 1");
    g_opt_gn_tail.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "srht_cols") {
    if (value < 0 || value > 1) return fail(TIK_EINVAL, "tik_set_option: srht_cols must be 0 or 1");
    g_opt_srht_cols.store(int(value));
    return TIK_OK;
  }
  if (std::string(name) == "chol_pivot_ulps") {
    if (value < 0 || value > (int64_t(1) << 53))
      return fail(TIK_EINVAL, "tik_set_option: chol_pivot_ulps must be 0..2^53");
    g_opt_pivot.store(value);
    return TIK_OK;
  }
  return fail(TIK_EINVAL, std::string("tik_set_option: unknown option ") + name);
}

int tik_get_option(const char* name, int64_t* value) {
  if (!name || !value) return fail(TIK_EINVAL, "tik_get_option: NULL argument");
  if (std::string(name) == "graph_chunk") {
    *value = option_chunk();
    return TIK_OK;
  }
  if (std::string(name) == "chol_pivot_ulps") {
    *value = option_pivot_ulps();
    return TIK_OK;
  }
  if (std::string(name) == "sparse_nnz") {
    *value = option_sparse_nnz();
    return TIK_OK;
  }
  if (std::string(name) == "cholqr_panels") {
    *value = option_cholqr_panels();
    return TIK_OK;
  }
  if (std::string(name) == "record_times") {
    *value = option_record_times() ? 1 : 0;
    return TIK_OK;
  }
  if (std::string(name) == "srht_cols") {
    *value = option_srht_cols();
    return TIK_OK;
  }
  if (std::string(name) == "gemm_n_tail") {
    *value = option_gemm_n_tail();
    return TIK_OK;
  }
  return fail(TIK_EINVAL, std::string("tik_get_option: unknown option ") + name);
}

int tik_prof_enable(int32_t on) {
  g_prof_on = on != 0;
  return TIK_OK;
}

int tik_prof_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& kv : g_prof)
    for (auto& e : kv.second.ev) {
      (void)hipEventSynchronize(e.second);
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  g_prof.clear();
  g_open.clear();
  return TIK_OK;
}

int tik_prof_query(const char* family, double* total_ms, int64_t* launches) {
  if (!family || !total_ms || !launches) return fail(TIK_EINVAL, "tik_prof_query: NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  auto it = g_prof.find(family);
  if (it == g_prof.end()) {
    *total_ms = 0.0;
    *launches = 0;
    return TIK_OK;
  }
  ProfFamily& f = it->second;
  for (auto& e : f.ev) {
    TIK_HIP(hipEventSynchronize(e.second));
    float ms = 0.f;
    TIK_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    f.done_ms += ms;
    f.done_n += 1;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  f.ev.clear();
  *total_ms = f.done_ms;
  *launches = f.done_n;
  return TIK_OK;
}

int tik_sketch_bytes(const tik_problem* p, int32_t nprob, int32_t embed, int32_t sketch_dtype,
                     const int64_t* s, size_t* bytes) {
  if (!bytes) return fail(TIK_EINVAL, "tik_sketch_bytes: bytes is NULL");
  TIK_TRY(sketch_validate(p, nprob, embed, sketch_dtype, s));
  Arena a;
  SketchPlan sp;
  TIK_TRY(sketch_plan(p, nprob, embed, sketch_dtype, s, a, sp));
  *bytes = a.used + 256;
  return TIK_OK;
}

int tik_sketch(const tik_problem* p, int32_t nprob, int32_t embed, int32_t sketch_dtype,
               const int64_t* s, uint64_t seed, void* dws, size_t dws_bytes, tik_stream_t stream,
               tik_sketch_t* out) {
  if (!out) return fail(TIK_EINVAL, "tik_sketch: out is NULL");
  *out = nullptr;
  TIK_TRY(sketch_validate(p, nprob, embed, sketch_dtype, s));
  size_t need = 0;
  TIK_TRY(tik_sketch_bytes(p, nprob, embed, sketch_dtype, s, &need));
  TIK_TRY(check_ws(dws, dws_bytes, need, "tik_sketch"));
  Arena a;
  a.base = static_cast<char*>(dws);
  a.cap = dws_bytes;
  SketchPlan sp;
  TIK_TRY(sketch_plan(p, nprob, embed, sketch_dtype, s, a, sp));
  Lanes lanes;
  TIK_TRY(lanes.fork(static_cast<hipStream_t>(stream), sp.lanes));
  for (int32_t k = 0; k < nprob; ++k) {
    const tik_problem& q = p[k];
    const int ln = k % lanes.n;
    hipStream_t st = lanes.at(k);
    // problem k draws from its own stream of the generator
    const uint64_t pseed = seed ^ (uint64_t(uint32_t(k)) * 0x9E3779B97F4A7C15ull);
    const int f32 = q.a_dtype == TIK_F32;
    if (embed == TIK_SPARSE) {
      TIK_TRY(launch_sparse_sketch(q.A, f32, q.m, q.n, q.lda, s[k], option_sparse_nnz(), pseed,
                                   sp.rows[ln], sp.Y[k], st));
    } else if (embed == TIK_SRHT) {
      const int kk = ilog2_ceil(q.m);
      const int bb = kk <= 13 ? kk : 13;
      int32_t* rows = sp.rows[ln];
      int32_t* bstart = rows + s[k];
      TIK_TRY(launch_srht_rows(pseed, kk, s[k], rows, bstart, bb, st));
      if (kk <= 13) {
        TIK_TRY(launch_srht_single(q.A, f32, q.m, q.n, q.lda, kk, pseed, rows, s[k], sp.Y[k], st));
      } else if (srht_cols_use(kk, q.n, s[k])) {
        TIK_TRY(launch_srht_cols(q.A, f32, q.m, q.n, q.lda, kk, bb, rows, s[k], sp.Y[k], st));
      } else {
        for (int64_t c0 = 0; c0 < q.n; c0 += sp.tcols) {
          const int64_t nc = std::min(sp.tcols, q.n - c0);
          TIK_TRY(launch_srht_twopass(q.A, f32, q.m, q.lda, c0, nc, kk, bb, rows, s[k], sp.T[ln],
                                      sp.Y[k], st));
        }
      }
    } else {
      const bool t = tall(q);
      const int64_t longdim = t ? q.m : q.n;
      const int64_t ncol = t ? q.n : q.m;
      const int64_t chunk = gauss_chunk(q, s[k], sketch_dtype);
      if (sketch_dtype == TIK_BF16 || sketch_dtype == TIK_F16) {
        const bool f16 = sketch_dtype == TIK_F16;
        if (f16) TIK_TRY(launch_col_pow2(q.A, f32, q.m, q.n, q.lda, sp.cscale[ln], st));
        for (int64_t r0 = 0; r0 < longdim; r0 += chunk) {
          const int64_t kc = std::min(chunk, longdim - r0);
          const int64_t ldx = gauss_pitch(kc, sketch_dtype);
          TIK_TRY(launch_gauss_gen(pseed, s[k], r0, kc, ldx, sp.Xc[ln], f16 ? 2 : 1, st));
          TIK_TRY(launch_sketch_gemm_bf16(sp.Xc[ln], s[k], kc, ldx, q.A, f32, q.lda, r0, ncol,
                                          t ? 0 : 1,
                                          sp.Yacc[ln], r0 == 0 ? 1 : 0, sp.Ypart[ln], sp.part_cap,
                                          st, f16 ? sp.cscale[ln] : nullptr));
        }
        if (f16)
          TIK_TRY(launch_f32_to_f64_cols(sp.Yacc[ln], sp.Y[k], s[k], ncol, sp.cscale[ln], st));
        else
          TIK_TRY(launch_f32_to_f64(sp.Yacc[ln], sp.Y[k], s[k] * ncol, st));
      } else {
        TIK_HIP(hipMemsetAsync(sp.Y[k], 0, size_t(s[k]) * size_t(ncol) * sizeof(double), st));
        for (int64_t r0 = 0; r0 < longdim; r0 += chunk) {
          const int64_t kc = std::min(chunk, longdim - r0);
          TIK_TRY(launch_gauss_gen(pseed, s[k], r0, kc, kc, sp.Xc[ln], 0, st));
          TIK_TRY(launch_sketch_gemm_f64(sp.Xc[ln], s[k], kc, q.A, f32, q.lda, r0, ncol, t ? 0 : 1,
                                         sp.Y[k], st));
        }
      }
    }
  }
  TIK_TRY(lanes.join());
  tik_sketch_s* h = new tik_sketch_s();
  h->probs.assign(p, p + nprob);
  h->embed = embed;
  h->sketch_dtype = sketch_dtype;
  h->s.assign(s, s + nprob);
  h->seed = seed;
  h->wide = !tall(p[0]);
  h->Y = sp.Y;
  h->yrows = sp.yrows;
  h->ycols = sp.ycols;
  *out = h;
  return TIK_OK;
}

int tik_sketch_data(tik_sketch_t sk, int32_t k, const double** Y, int64_t* rows, int64_t* cols) {
  if (!sk || !Y || !rows || !cols) return fail(TIK_EINVAL, "tik_sketch_data: NULL argument");
  if (k < 0 || k >= int32_t(sk->probs.size())) return fail(TIK_EINVAL, "tik_sketch_data: bad index");
  *Y = sk->Y[k];
  *rows = sk->yrows[k];
  *cols = sk->ycols[k];
  return TIK_OK;
}

void tik_sketch_free(tik_sketch_t sk) { delete sk; }

// ---------------------------------------------------------- preconditioner --
namespace {
struct PrecondPlan {
  std::vector<double*> Rinv;
  double* lams = nullptr;
  int32_t* notpd = nullptr;
  double* cnorm = nullptr;    // per problem
  int lanes = 1;
  double* colsum_l[kLanes] = {};   // per lane: scratch, kmax
  double* C_l[kLanes] = {};
  // Cholesky route: one job per (problem, lambda), sorted by size, largest first
  std::vector<CholJob> jobs;
  std::vector<int64_t> jobn;
  std::vector<int32_t> jobq;      // (problem, lambda) index k * N + i of each job
  CholJob* jobs_dev = nullptr;
  double* bp2 = nullptr;          // QR scratch of the breakdown fallback (largest problem)
  double* colsum = nullptr;   // scratch, kmax
  // low-rank route
  std::vector<double*> V, sigma, S;
  double* lr_scratch = nullptr;
  int32_t* perm = nullptr;
  int32_t* si = nullptr;
  unsigned int* cnt = nullptr;
};

constexpr int64_t kLowrankMaxS = 4096;

int precond_plan(tik_sketch_t sk, int32_t route, int32_t N, Arena& a, PrecondPlan& pp) {
  const int32_t np = int32_t(sk->probs.size());
  pp.Rinv.assign(size_t(np), nullptr);
  pp.V.assign(size_t(np), nullptr);
  pp.sigma.assign(size_t(np), nullptr);
  pp.S.assign(size_t(np), nullptr);
  int64_t kmax = 0, smax = 0;
  size_t scratch = 0;
  for (int32_t k = 0; k < np; ++k) {
    const int64_t kd = std::min(sk->probs[k].m, sk->probs[k].n);
    kmax = std::max(kmax, kd);
    if (route == TIK_ROUTE_CHOL) {
      pp.Rinv[k] = a.take<double>(size_t(N) * size_t(kd) * size_t(kd));
    } else {
      const int64_t s = sk->yrows[k];
      if (s > kd)
        return fail(TIK_EINVAL, "tik_precond: the low-rank route needs a sketch size s <= min(m, n) (problem " +
                                    std::to_string(k) + " has s = " + std::to_string(s) + ")");
      if (s > kLowrankMaxS)
        return fail(TIK_EINVAL, "tik_precond: the low-rank route supports s <= 4096");
      smax = std::max(smax, s);
      pp.V[k] = a.take<double>(size_t(kd) * size_t(s));
      pp.sigma[k] = a.take<double>(size_t(s));
      pp.S[k] = a.take<double>(size_t(N) * size_t(s));
      scratch = std::max(scratch, lowrank_scratch_doubles(kd, s));
    }
  }
  pp.lams = a.take<double>(size_t(np) * size_t(N));
  pp.notpd = a.take<int32_t>(size_t(np) * size_t(N));
  pp.cnorm = a.take<double>(size_t(np));
  pp.colsum = a.take<double>(size_t(kmax));
  if (route == TIK_ROUTE_CHOL) {
    pp.lanes = std::max(1, std::min<int>(kLanes, np));
    for (int l = 0; l < pp.lanes; ++l) {
      pp.colsum_l[l] = l == 0 ? pp.colsum : a.take<double>(size_t(kmax));
      pp.C_l[l] = a.take<double>(size_t(kmax) * size_t(kmax));
    }
    std::vector<int32_t> order(static_cast<size_t>(np));
    for (int32_t k = 0; k < np; ++k) order[size_t(k)] = k;
    auto kdim = [&](int32_t k) { return std::min(sk->probs[k].m, sk->probs[k].n); };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return kdim(x) > kdim(y); });
    pp.jobs.clear();
    pp.jobn.clear();
    pp.jobq.clear();
    size_t bp2 = 0;
    for (int32_t k : order) {
      const int64_t kd = kdim(k);
      bp2 = std::max(bp2, bp2_scratch_doubles(sk->yrows[size_t(k)], kd));
      for (int32_t i = 0; i < N; ++i) {
        CholJob j = {};
        j.R = pp.Rinv[size_t(k)] + size_t(i) * size_t(kd) * size_t(kd);
        j.Dinv = a.take<double>(size_t(cdiv(kd, 64)) * 64 * 64);
        j.notpd = pp.notpd + size_t(k) * size_t(N) + size_t(i);
        j.n = kd;
        j.dg = a.take<double>(size_t(kd));
        pp.jobs.push_back(j);
        pp.jobn.push_back(kd);
        pp.jobq.push_back(k * N + i);
      }
    }
    pp.jobs_dev = a.take<CholJob>(pp.jobs.size());
    pp.bp2 = a.take<double>(bp2);
  } else {
    pp.lr_scratch = a.take<double>(scratch);
    pp.perm = a.take<int32_t>(size_t(smax));
    pp.si = a.take<int32_t>(size_t(np) * size_t(N));
    pp.cnt = a.take<unsigned int>(1);
  }
  return TIK_OK;
}
}  // namespace

int tik_precond_bytes(tik_sketch_t sk, int32_t route, int32_t N, size_t* bytes) {
  if (!sk || !bytes) return fail(TIK_EINVAL, "tik_precond_bytes: NULL argument");
  if (route != TIK_ROUTE_CHOL && route != TIK_ROUTE_LOWRANK)
    return fail(TIK_EINVAL, "tik_precond_bytes: route must be TIK_ROUTE_CHOL or TIK_ROUTE_LOWRANK");
  if (N < 1) return fail(TIK_EINVAL, "tik_precond_bytes: N must be >= 1");
  Arena a;
  PrecondPlan pp;
  TIK_TRY(precond_plan(sk, route, N, a, pp));
  *bytes = a.used + 256;
  return TIK_OK;
}

// Algorithm 3 steps 4-7 (Algorithm 4 steps 4-7 for wide problems, whose
// sketch is stored transposed): SVD of the sketch, sd_hat per lambda
// (Section 3.1.2), s_i = min(s, ceil(alpha ceil(sd_hat_i))), S_i.
static int precond_lowrank(tik_sketch_t sk, const double* lambdas, int32_t N, double alpha,
                           PrecondPlan& pp, hipStream_t st, tik_precond_s* h) {
  const int32_t np = int32_t(sk->probs.size());
  h->sigma = pp.sigma;
  h->V = pp.V;
  h->S = pp.S;
  h->srank.assign(size_t(np), 0);
  h->si.assign(size_t(np) * N, 0);
  h->sdhat.assign(size_t(np) * N, 0.0);
  h->cnorm.assign(size_t(np), 0.0);
  h->status.assign(size_t(np) * N, TIK_ST_CONVERGED);
  h->lr_sweeps.assign(size_t(np), 0);
  for (int32_t k = 0; k < np; ++k) {
    const int64_t s = sk->yrows[k], kd = sk->ycols[k];
    h->srank[k] = s;
    int sweeps = 0;
    TIK_TRY(launch_lowrank_svd(sk->Y[k], s, kd, pp.V[k], pp.sigma[k], pp.lr_scratch, pp.cnt,
                               pp.perm, &sweeps, st));
    h->lr_sweeps[k] = sweeps;
    std::vector<double> sig(static_cast<size_t>(s));
    TIK_HIP(hipMemcpyAsync(sig.data(), pp.sigma[k], sizeof(double) * size_t(s),
                           hipMemcpyDeviceToHost, st));
    TIK_HIP(hipStreamSynchronize(st));
    bool finite = true;
    for (double v : sig) finite = finite && std::isfinite(v);
    h->cnorm[k] = finite && s > 0 ? sig[0] * sig[0] : std::nan("");
    for (int32_t i = 0; i < N; ++i) {
      const size_t q = size_t(k) * N + i;
      const double lam = lambdas[q];
      if (!finite) {
        h->status[q] = TIK_ST_NOTPD;
        h->sdhat[q] = std::nan("");
        h->si[q] = 0;
        continue;
      }
      double sd = 0.0;
      for (int64_t j = 0; j < s; ++j)
        if (sig[j] > 0.0) sd += 1.0 / (1.0 + lam / (sig[j] * sig[j]));
      h->sdhat[q] = sd;
      const double want = std::ceil(alpha * std::ceil(sd));
      h->si[q] = int32_t(std::min<double>(double(s), want));
    }
  }
  TIK_HIP(hipMemcpyAsync(pp.si, h->si.data(), sizeof(int32_t) * h->si.size(), hipMemcpyHostToDevice,
                         st));
  for (int32_t k = 0; k < np; ++k)
    TIK_TRY(launch_lowrank_S(pp.sigma[k], sk->yrows[k], pp.lams + size_t(k) * N, pp.si + size_t(k) * N,
                             N, pp.S[k], st));
  TIK_HIP(hipStreamSynchronize(st));   // h->si is host memory the copy reads
  return TIK_OK;
}

int tik_precond(tik_sketch_t sk, int32_t route, const double* lambdas, int32_t N, double alpha,
                void* dws, size_t dws_bytes, tik_stream_t stream, tik_precond_t* out,
                double* sd_hat, int32_t* status) {
  if (!out) return fail(TIK_EINVAL, "tik_precond: out is NULL");
  *out = nullptr;
  if (!sk) return fail(TIK_EINVAL, "tik_precond: sketch handle is NULL");
  if (!lambdas) return fail(TIK_EINVAL, "tik_precond: lambdas is NULL");
  if (route == TIK_ROUTE_LOWRANK && !(alpha >= 1.0 && std::isfinite(alpha)))
    return fail(TIK_EINVAL, "tik_precond: alpha must be finite and >= 1 for the low-rank route");
  const int32_t np = int32_t(sk->probs.size());
  for (int64_t q = 0; q < int64_t(np) * N; ++q)
    if (!(lambdas[q] > 0.0) || !std::isfinite(lambdas[q]))
      return fail(TIK_EINVAL, "tik_precond: every lambda must be positive and finite");
  size_t need = 0;
  TIK_TRY(tik_precond_bytes(sk, route, N, &need));
  TIK_TRY(check_ws(dws, dws_bytes, need, "tik_precond"));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Arena a;
  a.base = static_cast<char*>(dws);
  a.cap = dws_bytes;
  PrecondPlan pp;
  TIK_TRY(precond_plan(sk, route, N, a, pp));
  TIK_HIP(hipMemcpyAsync(pp.lams, lambdas, sizeof(double) * size_t(np) * size_t(N),
                         hipMemcpyHostToDevice, st));
  std::unique_ptr<tik_precond_s> h(new tik_precond_s());
  h->probs = sk->probs;
  h->wide = sk->wide;
  h->route = route;
  h->N = N;
  h->lams.assign(lambdas, lambdas + size_t(np) * N);
  for (int32_t k = 0; k < np; ++k) h->k.push_back(std::min(sk->probs[k].m, sk->probs[k].n));
  if (route == TIK_ROUTE_LOWRANK) {
    TIK_TRY(precond_lowrank(sk, lambdas, N, alpha, pp, st, h.get()));
  } else {
    TIK_HIP(hipMemsetAsync(pp.notpd, 0, sizeof(int32_t) * size_t(np) * size_t(N), st));
    Lanes lanes;
    TIK_TRY(lanes.fork(st, pp.lanes));
    for (int32_t k = 0; k < np; ++k) {
      const int64_t kd = std::min(sk->probs[k].m, sk->probs[k].n);
      const int ln = k % lanes.n;
      hipStream_t ls = lanes.at(k);
      // the problem's N lambda copies are written after the Gram: room for its partial products
      TIK_TRY(launch_syrk(sk->Y[k], sk->yrows[k], kd, sk->yrows[k], pp.C_l[ln], pp.Rinv[k], N, ls));
      TIK_TRY(launch_gram_norm_bound(pp.C_l[ln], kd, pp.colsum_l[ln], pp.cnorm + k, ls));
      TIK_TRY(launch_shift_copy(pp.C_l[ln], kd, pp.lams + size_t(k) * N, N, pp.Rinv[k], ls));
    }
    TIK_TRY(lanes.join());
    // every (problem, lambda) factored and inverted together, panel by panel
    const double floor = double(option_pivot_ulps()) * std::ldexp(1.0, -53);
    for (auto& j : pp.jobs) j.floor = floor;
    TIK_HIP(hipMemcpyAsync(pp.jobs_dev, pp.jobs.data(), pp.jobs.size() * sizeof(CholJob),
                           hipMemcpyHostToDevice, st));
    if (floor > 0.0)
      TIK_TRY(launch_save_diag(pp.jobs_dev, int32_t(pp.jobs.size()), pp.jobn.empty() ? 0 : pp.jobn[0], st));
    TIK_TRY(launch_chol_inv_jobs(pp.jobs_dev, pp.jobn.data(), int32_t(pp.jobs.size()), st));
    std::vector<int32_t> bad(size_t(np) * size_t(N), 0);
    std::vector<double> cn(size_t(np), 0.0);
    TIK_HIP(hipMemcpyAsync(bad.data(), pp.notpd, sizeof(int32_t) * bad.size(),
                           hipMemcpyDeviceToHost, st));
    TIK_HIP(hipMemcpyAsync(cn.data(), pp.cnorm, sizeof(double) * cn.size(), hipMemcpyDeviceToHost, st));
    TIK_HIP(hipStreamSynchronize(st));
    h->Rinv = pp.Rinv;
    h->cnorm = cn;
    h->status.resize(bad.size());
    h->qr.assign(bad.size(), 0);
    for (size_t q = 0; q < bad.size(); ++q) h->status[q] = bad[q] ? TIK_ST_NOTPD : TIK_ST_CONVERGED;
    h->sdhat.assign(bad.size(), std::nan(""));
    // Breakdown fallback (the BP2 preconditioner of Section 4.1): for every
    // (problem, lambda) whose Cholesky factorization broke down, R from the
    // Householder QR of [Y; sqrt(lambda) I], which never forms the Gram matrix,
    // then its inverse; all of them inverted in one batched pass
    std::vector<CholJob> fb;
    std::vector<int64_t> fbn;
    std::vector<int32_t> fbq;
    for (size_t jx = 0; jx < pp.jobs.size(); ++jx) {
      const int32_t q = pp.jobq[jx];
      if (!bad[size_t(q)]) continue;
      const int32_t k = q / N;
      const double lam = h->lams[size_t(q)];
      if (!(lam > 0.0) || !std::isfinite(lam)) continue;
      CholJob j = pp.jobs[jx];
      TIK_TRY(launch_bp2_r(sk->Y[size_t(k)], sk->yrows[size_t(k)], j.n, lam, j.R, pp.bp2, st));
      j.given = 1;
      j.dg = nullptr;
      fb.push_back(j);
      fbn.push_back(j.n);
      fbq.push_back(q);
    }
    if (!fb.empty()) {
      // jobs of one problem are contiguous and the table is sorted by size:
      // the fallback subset keeps that order
      TIK_HIP(hipMemsetAsync(pp.notpd, 0, sizeof(int32_t) * size_t(np) * size_t(N), st));
      TIK_HIP(hipMemcpyAsync(pp.jobs_dev, fb.data(), fb.size() * sizeof(CholJob), hipMemcpyHostToDevice, st));
      TIK_TRY(launch_chol_inv_jobs(pp.jobs_dev, fbn.data(), int32_t(fb.size()), st, true));
      TIK_HIP(hipMemcpyAsync(bad.data(), pp.notpd, sizeof(int32_t) * bad.size(),
                             hipMemcpyDeviceToHost, st));
      TIK_HIP(hipStreamSynchronize(st));
      for (int32_t q : fbq)
        if (!bad[size_t(q)]) {
          h->status[size_t(q)] = TIK_ST_CONVERGED;
          h->qr[size_t(q)] = 1;
        }
    }
  }
  if (status) {
    std::memcpy(status, h->status.data(), sizeof(int32_t) * h->status.size());
    for (size_t q = 0; q < h->qr.size(); ++q)
      if (h->qr[q]) status[q] = TIK_ST_QR;
  }
  if (sd_hat) std::memcpy(sd_hat, h->sdhat.data(), sizeof(double) * h->sdhat.size());
  *out = h.release();
  return TIK_OK;
}

int tik_precond_data(tik_precond_t pc, int32_t k, int32_t i, const double** data, int64_t* dim,
                     int64_t* rank) {
  if (!pc || !data || !dim || !rank) return fail(TIK_EINVAL, "tik_precond_data: NULL argument");
  if (k < 0 || k >= int32_t(pc->probs.size()) || i < 0 || i >= pc->N)
    return fail(TIK_EINVAL, "tik_precond_data: index out of range");
  const int64_t kd = pc->k[k];
  *dim = kd;
  if (pc->route == TIK_ROUTE_CHOL) {
    *data = pc->Rinv[k] + int64_t(i) * kd * kd;
    *rank = kd;
  } else {
    *data = pc->V[k];
    *rank = pc->si[size_t(k) * pc->N + i];
  }
  return TIK_OK;
}

int tik_precond_sigma(tik_precond_t pc, int32_t k, const double** sigma, int64_t* count) {
  if (!pc || !sigma || !count) return fail(TIK_EINVAL, "tik_precond_sigma: NULL argument");
  if (k < 0 || k >= int32_t(pc->probs.size()))
    return fail(TIK_EINVAL, "tik_precond_sigma: index out of range");
  if (pc->route != TIK_ROUTE_LOWRANK)
    return fail(TIK_EINVAL, "tik_precond_sigma: only the low-rank route keeps singular values");
  *sigma = pc->sigma[k];
  *count = pc->srank[k];
  return TIK_OK;
}

int tik_precond_sweeps(tik_precond_t pc, int32_t k, int32_t* sweeps) {
  if (!pc || !sweeps) return fail(TIK_EINVAL, "tik_precond_sweeps: NULL argument");
  if (k < 0 || k >= int32_t(pc->probs.size()))
    return fail(TIK_EINVAL, "tik_precond_sweeps: index out of range");
  if (pc->route != TIK_ROUTE_LOWRANK)
    return fail(TIK_EINVAL, "tik_precond_sweeps: only the low-rank route computes an SVD");
  *sweeps = pc->lr_sweeps[size_t(k)];
  return TIK_OK;
}

void tik_precond_free(tik_precond_t pc) { delete pc; }

// ------------------------------------------------------------------ solve --
static int lsqr_validate(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode) {
  TIK_TRY(validate_problems(p, nprob, "tik_lsqr_batch"));
  if (!pc) return fail(TIK_EINVAL, "tik_lsqr_batch: preconditioner handle is NULL");
  if (int32_t(pc->probs.size()) != nprob)
    return fail(TIK_EINVAL, "tik_lsqr_batch: problem count differs from the preconditioner's");
  for (int32_t k = 0; k < nprob; ++k) {
    const tik_problem &a = p[k], &b = pc->probs[k];
    if (a.m != b.m || a.n != b.n || a.lda != b.lda || a.A != b.A || a.b != b.b ||
        a.a_dtype != b.a_dtype)
      return fail(TIK_EINVAL, "tik_lsqr_batch: problem " + std::to_string(k) +
                                  " differs from the one the sketch was built from");
  }
  if (mode != TIK_PLAIN_F64_PER_LAMBDA && mode != TIK_F64_BATCHED && mode != TIK_MIXED_BATCHED)
    return fail(TIK_EINVAL, "tik_lsqr_batch: unknown mode");

  return TIK_OK;
}

int tik_lsqr_batch_bytes(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                         size_t* bytes) {
  if (!bytes) return fail(TIK_EINVAL, "tik_lsqr_batch_bytes: bytes is NULL");
  TIK_TRY(lsqr_validate(p, nprob, pc, mode));
  return lsqr_bytes(p, nprob, pc, mode, bytes);
}

static int lsqr_args(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                     double tol, int32_t maxit, double* const* X) {
  TIK_TRY(lsqr_validate(p, nprob, pc, mode));
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(TIK_EINVAL, "tik_lsqr_batch: tol must be > 0");
  if (maxit < 1) return fail(TIK_EINVAL, "tik_lsqr_batch: maxit must be >= 1");
  if (!X) return fail(TIK_EINVAL, "tik_lsqr_batch: X is NULL");
  for (int32_t k = 0; k < nprob; ++k)
    if (!X[k]) return fail(TIK_EINVAL, "tik_lsqr_batch: X[" + std::to_string(k) + "] is NULL");
  return TIK_OK;
}

int tik_lsqr_batch_static(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                          double tol, int32_t maxit, double* const* X, int32_t* iters,
                          int32_t* status, double* relres, tik_stream_t stream) {
  TIK_TRY(lsqr_args(p, nprob, pc, mode, tol, maxit, X));
  size_t need = 0;
  TIK_TRY(lsqr_bytes(p, nprob, pc, mode, &need));
  if (need > kStaticBytes)
    return fail(TIK_ENOTSUP, "tik_lsqr_batch_static: this solve needs " + std::to_string(need) +
                                 " bytes of workspace, more than the " + std::to_string(kStaticBytes) +
                                 " bytes of the static workspace; use tik_lsqr_batch");
  void* ws = nullptr;
  TIK_TRY(scratch_address(&ws));
  NoAllocScope guard;
  g_split32 = g_split64 = 0;
  times_reset(option_record_times() ? int64_t(nprob) * pc->N : 0);
  return lsqr_run(p, nprob, pc, mode, tol, maxit, X, iters, status, relres, ws, kStaticBytes,
                  static_cast<hipStream_t>(stream));
}

int tik_lsqr_batch(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t mode,
                   double tol, int32_t maxit, double* const* X, int32_t* iters, int32_t* status,
                   double* relres, void* dws, size_t dws_bytes, tik_stream_t stream) {
  TIK_TRY(lsqr_args(p, nprob, pc, mode, tol, maxit, X));
  size_t need = 0;
  TIK_TRY(lsqr_bytes(p, nprob, pc, mode, &need));
  TIK_TRY(check_ws(dws, dws_bytes, need, "tik_lsqr_batch"));
  g_split32 = g_split64 = 0;
  times_reset(option_record_times() ? int64_t(nprob) * pc->N : 0);
  return lsqr_run(p, nprob, pc, mode, tol, maxit, X, iters, status, relres, dws, dws_bytes,
                  static_cast<hipStream_t>(stream));
}

// --------------------------------------------------------------- L-curve --
int tik_lcurve_bytes(const tik_problem* p, int32_t nprob, size_t* bytes) {
  if (!bytes) return fail(TIK_EINVAL, "tik_lcurve_bytes: bytes is NULL");
  TIK_TRY(validate_problems(p, nprob, "tik_lcurve"));
  return lcurve_bytes(p, nprob, bytes);
}

int tik_lcurve(const tik_problem* p, int32_t nprob, int32_t N, double* const* X, double* xnorm,
               double* rnorm, void* dws, size_t dws_bytes, tik_stream_t stream) {
  TIK_TRY(validate_problems(p, nprob, "tik_lcurve"));
  if (N < 1) return fail(TIK_EINVAL, "tik_lcurve: N must be >= 1");
  if (!X) return fail(TIK_EINVAL, "tik_lcurve: X is NULL");
  for (int32_t k = 0; k < nprob; ++k)
    if (!X[k]) return fail(TIK_EINVAL, "tik_lcurve: X[" + std::to_string(k) + "] is NULL");
  if (!xnorm && !rnorm) return fail(TIK_EINVAL, "tik_lcurve: both outputs are NULL");
  size_t need = 0;
  TIK_TRY(lcurve_bytes(p, nprob, &need));
  TIK_TRY(check_ws(dws, dws_bytes, need, "tik_lcurve"));
  return lcurve_run(p, nprob, N, X, xnorm, rnorm, dws, dws_bytes, static_cast<hipStream_t>(stream));
}

int tik_lcurve_corner(const double* lambdas, const double* xnorm, const double* rnorm, int32_t N,
                      int32_t* corner, double* curvature) {
  if (!lambdas || !xnorm || !rnorm || !corner)
    return fail(TIK_EINVAL, "tik_lcurve_corner: NULL argument");
  if (N < 3) return fail(TIK_EINVAL, "tik_lcurve_corner: needs at least 3 lambdas");
  std::vector<int> ord(static_cast<size_t>(N));
  for (int j = 0; j < N; ++j) ord[size_t(j)] = j;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lambdas[a] < lambdas[b]; });
  for (int j = 0; j < N; ++j) {
    const int i = ord[size_t(j)];
    if (!(lambdas[i] > 0.0) || !std::isfinite(lambdas[i]))
      return fail(TIK_EINVAL, "tik_lcurve_corner: lambdas must be positive and finite");
    if (j > 0 && !(lambdas[i] > lambdas[ord[size_t(j - 1)]]))
      return fail(TIK_EINVAL, "tik_lcurve_corner: lambdas must be distinct");
    if (!(xnorm[i] > 0.0) || !(rnorm[i] > 0.0) || !std::isfinite(xnorm[i]) || !std::isfinite(rnorm[i]))
      return fail(TIK_EINVAL, "tik_lcurve_corner: norms must be positive and finite");
  }
  // the curve (log ||A x - b||, log ||x||) as a function of t = log lambda,
  // lambda increasing; signed curvature (x' y'' - x'' y') / (x'^2 + y'^2)^(3/2)
  // with second-order three-point differences on the uneven grid; the corner
  // is its largest value over the interior points (Hansen's criterion)
  const size_t nn = static_cast<size_t>(N);
  std::vector<double> t(nn), cx(nn), cy(nn);
  for (int j = 0; j < N; ++j) {
    const int i = ord[size_t(j)];
    t[size_t(j)] = std::log(lambdas[i]);
    cx[size_t(j)] = std::log(rnorm[i]);
    cy[size_t(j)] = std::log(xnorm[i]);
  }
  if (curvature)
    for (int j = 0; j < N; ++j) curvature[j] = std::nan("");
  int best = -1;
  double kbest = 0.0;
  for (int j = 1; j + 1 < N; ++j) {
    const double h1 = t[size_t(j)] - t[size_t(j - 1)], h2 = t[size_t(j + 1)] - t[size_t(j)];
    const double wm = -h2 / (h1 * (h1 + h2)), w0 = (h2 - h1) / (h1 * h2), wp = h1 / (h2 * (h1 + h2));
    const double vm = 2.0 / (h1 * (h1 + h2)), v0 = -2.0 / (h1 * h2), vp = 2.0 / (h2 * (h1 + h2));
    const double x1 = wm * cx[size_t(j - 1)] + w0 * cx[size_t(j)] + wp * cx[size_t(j + 1)];
    const double y1 = wm * cy[size_t(j - 1)] + w0 * cy[size_t(j)] + wp * cy[size_t(j + 1)];
    const double x2 = vm * cx[size_t(j - 1)] + v0 * cx[size_t(j)] + vp * cx[size_t(j + 1)];
    const double y2 = vm * cy[size_t(j - 1)] + v0 * cy[size_t(j)] + vp * cy[size_t(j + 1)];
    const double k = (x1 * y2 - x2 * y1) / std::pow(x1 * x1 + y1 * y1, 1.5);
    if (curvature) curvature[ord[size_t(j)]] = k;
    if (std::isfinite(k) && (best < 0 || k > kbest)) {
      best = ord[size_t(j)];
      kbest = k;
    }
  }
  if (best < 0) return fail(TIK_EINVAL, "tik_lcurve_corner: the curve has no finite curvature");
  *corner = best;
  return TIK_OK;
}

// ------------------------------------------------------------ autotuner --
int tik_tune_bytes(const tik_problem* p, int32_t nprob, tik_precond_t pc, size_t* bytes) {
  if (!bytes) return fail(TIK_EINVAL, "tik_tune_bytes: bytes is NULL");
  TIK_TRY(lsqr_validate(p, nprob, pc, TIK_F64_BATCHED));
  return tune_bytes(p, nprob, pc, bytes);
}

int tik_tune(const tik_problem* p, int32_t nprob, tik_precond_t pc, int32_t iters, void* dws,
             size_t dws_bytes, tik_stream_t stream, int32_t* best, double* best_ms, double* default_ms) {
  TIK_TRY(lsqr_validate(p, nprob, pc, TIK_F64_BATCHED));
  if (iters < 2 || iters > 1000) return fail(TIK_EINVAL, "tik_tune: iters must be 2..1000");
  size_t need = 0;
  TIK_TRY(tune_bytes(p, nprob, pc, &need));
  TIK_TRY(check_ws(dws, dws_bytes, need, "tik_tune"));
  int b[3] = {0, 0, 0};
  TIK_TRY(tune_class(p, nprob, pc, iters, dws, dws_bytes, static_cast<hipStream_t>(stream), b, best_ms,
                     default_ms));
  if (best)
    for (int i = 0; i < 3; ++i) best[i] = b[i];
  return TIK_OK;
}

int tik_tune_save(const char* path) {
  if (!path) return fail(TIK_EINVAL, "tik_tune_save: path is NULL");
  return tiles_save(path);
}

int tik_tune_load(const char* path, int32_t* loaded) {
  if (!path) return fail(TIK_EINVAL, "tik_tune_load: path is NULL");
  int n = 0;
  TIK_TRY(tiles_load(path, &n));
  if (loaded) *loaded = n;
  return TIK_OK;
}

int tik_last_tiles(char* buf, int32_t len) {
  if (!buf || len < 1) return fail(TIK_EINVAL, "tik_last_tiles: empty buffer");
  const std::string& t = last_tile();
  const size_t n = std::min(t.size(), size_t(len - 1));
  std::memcpy(buf, t.data(), n);
  buf[n] = 0;
  return TIK_OK;
}

int tik_lsqr_times(double* ms, int64_t count) {
  if (!ms || count < 0) return fail(TIK_EINVAL, "tik_lsqr_times: NULL or negative");
  if (int64_t(g_times.size()) != count)
    return fail(TIK_EINVAL, "tik_lsqr_times: count must equal nprob * N of the last tik_lsqr_batch call "
                            "made with record_times = 1");
  std::copy(g_times.begin(), g_times.end(), ms);
  return TIK_OK;
}

int tik_lsqr_info(int32_t* fp32, int32_t* fp64) {
  if (!fp32 || !fp64) return fail(TIK_EINVAL, "tik_lsqr_info: NULL argument");
  last_split(fp32, fp64);
  return TIK_OK;
}

}  // extern "C"
